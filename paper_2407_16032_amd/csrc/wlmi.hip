// Host orchestration and C ABI of the BDIM projection step (see include/wlmi.h).
//
// One time step (paper, numerical-methods section) is enqueued as:
//   [measure]  flux(u0) -> f~  bdim -> u*  [exit]  bc  project(w=1)  bc
//   flux(u') -> f~  bdim(avg) -> u**  bc  project(w=1/2)  bc  cfl
// with the projection = div/residual, multigrid V(0,1) cycles with a PCG(k)
// smoother on every level plus a fine PCG(k), and the velocity update.
// Velocity ping-pongs between two buffers so u0 never needs a copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "wlmi.h"
#include "wl_kernels.hpp"
#include "wl_pgnet.hpp"
#include "wl_adjoint.hpp"

using namespace wl;

// Scratch of the allocation-free force entry point (wl_forces_static): the 11
// per-block partials of the force sums (kGridStride blocks at most, the grid
// of k_forces) and their 11 totals.  Each GPU the library runs on holds one copy
// until the process ends; every call on that GPU shares it.
constexpr int kScratchRows = 11;
constexpr int kScratchDoubles = kScratchRows * kGridStride + 16;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_err;

wl_status fail(wl_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define WL_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(WL_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int blocks_for(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > kGridStride) b = kGridStride;
  return (int)b;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// workspace plan
// ---------------------------------------------------------------------------
struct LevelPlan {
  int n[3];
  int px, py, pz;
  int64_t elems;  // px*py*pz
  int64_t alloc;  // elems + front padding (16-element multiple)
};

struct Plan {
  int ndim = 0, nlev = 0;
  size_t esize = 4;
  LevelPlan lev[kMaxLevels];
  int64_t grid_cnt[kMaxParts] = {};  // samples of each gridded part (0: not gridded)
  bool grid_vel[kMaxParts] = {};     // with a sampled velocity
  size_t bytes = 0;
};

wl_status validate_and_default(const wl_sim_desc* in, wl_sim_desc* d) {
  if (!in) return fail(WL_ERR_INVALID_ARG, "desc is NULL");
  *d = *in;
  if (d->ndim != 2 && d->ndim != 3) return fail(WL_ERR_INVALID_ARG, "ndim must be 2 or 3");
  if (d->ndim == 2) d->n[2] = 1;
  for (int a = 0; a < d->ndim; ++a)
    if (d->n[a] < 4 || d->n[a] > (1 << 20)) return fail(WL_ERR_INVALID_ARG, "n[a] must be in [4, 2^20]");
  if (d->prec != WL_F32 && d->prec != WL_F64) return fail(WL_ERR_INVALID_ARG, "prec must be WL_F32 or WL_F64");
  if (!(d->nu >= 0.0) || !std::isfinite(d->nu)) return fail(WL_ERR_INVALID_ARG, "nu must be finite and >= 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->U[a])) return fail(WL_ERR_INVALID_ARG, "U must be finite");
  if (d->L == 0.0) d->L = 1.0;
  if (!(d->L > 0.0) || !std::isfinite(d->L)) return fail(WL_ERR_INVALID_ARG, "L must be finite and > 0");
  if (d->eps == 0.0) d->eps = 1.0;
  if (d->dt0 == 0.0) d->dt0 = 0.25;
  if (d->dt_max == 0.0) d->dt_max = 10.0;
  if (d->cfl_nu_coef == 0.0) d->cfl_nu_coef = 5.0;
  if (d->mg_tol == 0.0) d->mg_tol = 1e-6;
  if (d->mg_itmax == 0) d->mg_itmax = 32;
  if (d->pcg_iters == 0) d->pcg_iters = 6;
  if (!(d->eps > 0.0) || !(d->dt0 > 0.0) || !(d->dt_max > 0.0) || !(d->mg_tol > 0.0) || d->mg_itmax < 1)
    return fail(WL_ERR_INVALID_ARG, "eps, dt0, dt_max, mg_tol must be > 0 and mg_itmax >= 1");
  if (d->pcg_iters < 1 || d->pcg_iters > kMaxPcg) return fail(WL_ERR_INVALID_ARG, "pcg_iters must be in [1, 15]");
  if (d->solver_path < 0 || d->solver_path > 3) return fail(WL_ERR_INVALID_ARG, "solver_path must be in [0, 3]");
  if (d->reduce_mode < 0 || d->reduce_mode > 2) return fail(WL_ERR_INVALID_ARG, "reduce_mode must be in [0, 2]");
  if (d->blend_mode < 0 || d->blend_mode > 1) return fail(WL_ERR_INVALID_ARG, "blend_mode must be 0 or 1");
  if (d->vcycle_graph < 0 || d->vcycle_graph > 2) return fail(WL_ERR_INVALID_ARG, "vcycle_graph must be in [0, 2]");
  if (d->convective_exit) {
    if (d->periodic_mask & 1u) return fail(WL_ERR_INVALID_ARG, "convective exit needs a non-periodic x axis");
    if (d->U[0] == 0.0) return fail(WL_ERR_INVALID_ARG, "convective exit needs U[0] != 0");
  }
  return WL_OK;
}

// ---------------------------------------------------------------------------
// bodies: a chain of parts (see wl_body_desc)
// ---------------------------------------------------------------------------
int64_t grid_count(const wl_body_desc& b, int D) {
  int64_t c = 1;
  for (int a = 0; a < D; ++a) c *= b.grid_n[a];
  return c;
}

// copies of the parts of a body (next cleared); an empty list for no body
wl_status collect_parts(const wl_body_desc* b, std::vector<wl_body_desc>& out) {
  out.clear();
  if (!b || b->kind == WL_BODY_NONE) return WL_OK;
  for (const wl_body_desc* q = b; q; q = q->next) {
    if ((int)out.size() == kMaxParts) return fail(WL_ERR_INVALID_ARG, "a body has at most 4 parts");
    out.push_back(*q);
    out.back().next = nullptr;
  }
  return WL_OK;
}

bool part_needs_general(const wl_body_desc& p) {
  return p.kind == WL_BODY_PLANE || p.shell != 0.0 || p.scale_amp[0] != 0.0 || p.scale_amp[1] != 0.0 ||
         p.scale_amp[2] != 0.0;
}
bool part_moving(const wl_body_desc& p) {
  return p.heave_amp != 0.0 || p.pitch_amp != 0.0 || p.spin_omega != 0.0 || p.velocity[0] != 0.0 ||
         p.velocity[1] != 0.0 || p.velocity[2] != 0.0 ||
         (p.freq != 0.0 && (p.scale_amp[0] != 0.0 || p.scale_amp[1] != 0.0 || p.scale_amp[2] != 0.0));
}
bool parts_general(const std::vector<wl_body_desc>& ps) {
  if (ps.size() > 1) return true;
  for (const auto& p : ps)
    if (part_needs_general(p)) return true;
  return false;
}

void heave_unit(const wl_body_desc& b, double e[3]) {
  const double m = std::sqrt(b.heave_dir[0] * b.heave_dir[0] + b.heave_dir[1] * b.heave_dir[1] +
                             b.heave_dir[2] * b.heave_dir[2]);
  for (int k = 0; k < 3; ++k) e[k] = m == 0.0 ? (k == 1 ? 1.0 : 0.0) : b.heave_dir[k] / m;
}

// extreme scales of a part's map over its cycle
double scale_min(const wl_body_desc& b) {
  const double a = std::max(std::fabs(b.scale_amp[0]), std::max(std::fabs(b.scale_amp[1]), std::fabs(b.scale_amp[2])));
  return 1.0 - a;
}
double scale_max(const wl_body_desc& b) {
  const double a = std::max(std::fabs(b.scale_amp[0]), std::max(std::fabs(b.scale_amp[1]), std::fabs(b.scale_amp[2])));
  return 1.0 + a;
}

// body-frame radius that holds the part's shape around the body-frame origin
// (infinite for a plane)
double shape_radius(const wl_body_desc& b, int D) {
  double r = 0.0;
  if (b.kind == WL_BODY_SPHERE) {
    r = b.radius;
  } else if (b.kind == WL_BODY_BOX) {
    double s = 0;
    for (int a = 0; a < D; ++a) s += b.half_extent[a] * b.half_extent[a];
    r = std::sqrt(s);
  } else if (b.kind == WL_BODY_GRID_SDF) {
    double s = 0;
    for (int a = 0; a < D; ++a) {
      const double lo = b.grid_origin[a], hi = b.grid_origin[a] + (b.grid_n[a] - 1) * b.grid_h;
      const double m = std::max(std::fabs(lo), std::fabs(hi));
      s += m * m;
    }
    r = std::sqrt(s);
  } else {
    return INFINITY;
  }
  return r + std::max(0.0, b.shell);
}

// Pivot position of a part at time t (heave included unless `heave` is false).
void part_pivot(const wl_body_desc& b, double t, double P[3], bool heave = true) {
  const double w = 2.0 * M_PI * b.freq;
  double eh[3];
  heave_unit(b, eh);
  const double hv = heave ? b.heave_amp * std::sin(w * t + b.phase_h) : 0.0;
  for (int k = 0; k < 3; ++k) P[k] = b.center[k] + b.velocity[k] * t + hv * eh[k] + b.pivot_offset[k];
}

// World interval per axis that holds every point of the body where measure can
// set a coefficient (d < 2 + eps), plus `margin` cells, at time t: per part a
// ball around its pivot (the heave's whole excursion when `cycle`), combined
// as the parts combine.  lo > hi on an axis: empty; +-inf: unbounded.
void body_extent(const std::vector<wl_body_desc>& ps, int D, double eps, double t, bool cycle, double margin,
                 double lo[3], double hi[3]) {
  for (size_t k = 0; k < ps.size(); ++k) {
    const wl_body_desc& b = ps[k];
    double plo[3], phi[3];
    const double rb = shape_radius(b, D);
    double po = 0;
    for (int a = 0; a < D; ++a) po += b.pivot_offset[a] * b.pivot_offset[a];
    const double reach = (rb + std::sqrt(po) + (2.0 + eps) * scale_max(b)) / scale_min(b) + margin;
    double P[3];
    part_pivot(b, t, P, !cycle);
    double eh[3];
    heave_unit(b, eh);
    for (int a = 0; a < 3; ++a) {
      // over a whole cycle the heave moves the pivot by up to its amplitude either way
      const double ex = cycle ? std::fabs(b.heave_amp * eh[a]) : 0.0;
      plo[a] = std::isinf(reach) ? -INFINITY : P[a] - reach - ex;
      phi[a] = std::isinf(reach) ? INFINITY : P[a] + reach + ex;
    }
    for (int a = 0; a < 3; ++a) {
      if (k == 0 || b.op == WL_OP_UNION) {
        lo[a] = k == 0 ? plo[a] : std::min(lo[a], plo[a]);
        hi[a] = k == 0 ? phi[a] : std::max(hi[a], phi[a]);
      } else if (b.op == WL_OP_INTERSECT) {
        lo[a] = std::max(lo[a], plo[a]);
        hi[a] = std::min(hi[a], phi[a]);
      }  // subtract: the body stays inside the parts before it
    }
  }
}

wl_status validate_part(const wl_sim_desc& d, const wl_body_desc& b, bool first) {
  if (b.kind < WL_BODY_SPHERE || b.kind > WL_BODY_PLANE)
    return fail(WL_ERR_UNSUPPORTED, "body kind not supported (sphere, box, gridded SDF and plane are)");
  const double vals[] = {b.radius, b.heave_amp, b.pitch_amp, b.freq, b.phase_h, b.phase_p, b.spin_omega, b.phase_s,
                         b.shell, b.grid_h};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(WL_ERR_INVALID_ARG, "body parameters must be finite");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(b.center[k]) || !std::isfinite(b.half_extent[k]) || !std::isfinite(b.pivot_offset[k]) ||
        !std::isfinite(b.velocity[k]) || !std::isfinite(b.heave_dir[k]) || !std::isfinite(b.scale_amp[k]) ||
        !std::isfinite(b.normal[k]) || !std::isfinite(b.grid_origin[k]))
      return fail(WL_ERR_INVALID_ARG, "body parameters must be finite");
  if (!first && (b.op < WL_OP_UNION || b.op > WL_OP_SUBTRACT))
    return fail(WL_ERR_INVALID_ARG, "op must be WL_OP_UNION, WL_OP_INTERSECT or WL_OP_SUBTRACT");
  if (b.kind == WL_BODY_SPHERE && !(b.radius > 0.0)) return fail(WL_ERR_INVALID_ARG, "sphere radius must be > 0");
  if (b.kind == WL_BODY_BOX)
    for (int a = 0; a < d.ndim; ++a)
      if (!(b.half_extent[a] > 0.0)) return fail(WL_ERR_INVALID_ARG, "box half extents must be > 0");
  if (b.kind == WL_BODY_PLANE) {
    double m = 0;
    for (int a = 0; a < d.ndim; ++a) m += b.normal[a] * b.normal[a];
    if (!(m > 0.0)) return fail(WL_ERR_INVALID_ARG, "plane normal must be nonzero");
  }
  if (b.kind == WL_BODY_GRID_SDF) {
    if (!b.sdf_grid) return fail(WL_ERR_INVALID_ARG, "gridded SDF needs sdf_grid");
    if (!(b.grid_h > 0.0)) return fail(WL_ERR_INVALID_ARG, "grid_h must be > 0");
    for (int a = 0; a < d.ndim; ++a)
      if (b.grid_n[a] < 2 || b.grid_n[a] > 4096) return fail(WL_ERR_INVALID_ARG, "grid_n[a] must be in [2, 4096]");
    if (grid_count(b, d.ndim) > (int64_t(1) << 26)) return fail(WL_ERR_INVALID_ARG, "sdf_grid has more than 2^26 samples");
  } else if (b.vel_grid) {
    return fail(WL_ERR_INVALID_ARG, "vel_grid needs a gridded SDF part");
  }
  if (b.shell < 0.0) return fail(WL_ERR_INVALID_ARG, "shell must be >= 0");
  for (int a = 0; a < 3; ++a)
    if (!(std::fabs(b.scale_amp[a]) < 0.9)) return fail(WL_ERR_INVALID_ARG, "|scale_amp| must be < 0.9");
  return WL_OK;
}

// the body's reach (every point where measure can set a coefficient) must stay at
// least 3 cells inside the non-periodic domain faces at time t
wl_status check_reach(const wl_sim_desc& d, const std::vector<wl_body_desc>& ps, double t, bool cycle) {
  if (ps.empty()) return WL_OK;
  double lo[3], hi[3];
  body_extent(ps, d.ndim, d.eps, t, cycle, 0.0, lo, hi);
  for (int a = 0; a < d.ndim; ++a) {
    if (d.periodic_mask & (1u << a)) continue;
    if (lo[a] > hi[a]) continue;  // empty body
    if (std::isinf(lo[a]) || std::isinf(hi[a]))
      return fail(WL_ERR_INVALID_ARG, "the body is unbounded (a plane must be subtracted or intersected)");
    if (lo[a] < 3.0 || hi[a] > double(d.n[a]) - 3.0)
      return fail(WL_ERR_INVALID_ARG, "body must stay at least 3 cells from non-periodic boundaries");
  }
  return WL_OK;
}

wl_status validate_body(const wl_sim_desc& d, const wl_body_desc* b) {
  std::vector<wl_body_desc> ps;
  wl_status s = collect_parts(b, ps);
  if (s != WL_OK) return s;
  for (size_t k = 0; k < ps.size(); ++k)
    if ((s = validate_part(d, ps[k], k == 0)) != WL_OK) return s;
  return check_reach(d, ps, 0.0, true);
}

// FP64 doubles of the workspace that hold a body's sampled parts
int64_t body_grid_doubles(const std::vector<wl_body_desc>& ps, int D) {
  int64_t n = 0;
  for (const auto& p : ps)
    if (p.kind == WL_BODY_GRID_SDF) n += grid_count(p, D) * (1 + D + (p.vel_grid ? D : 0));
  return n;
}

// learned-guess buffer sizes: the whole padded grid (inference) and one crop box
constexpr int kPgRing = 64;     // crops kept for training
constexpr int kPgWaves = 1024;  // waves of the weight-gradient kernels (256 blocks)
struct PgSizes {
  int64_t Pd, Pc;
  int cn[3];
};
PgSizes pg_sizes(const Plan& P) {
  PgSizes S;
  S.Pd = (int64_t)(P.lev[0].n[0] + 2) * (P.lev[0].n[1] + 2) * (P.lev[0].n[2] + 2);
  S.Pc = 1;
  for (int a = 0; a < 3; ++a) {
    S.cn[a] = std::min(kPgCrop, P.lev[0].n[a]);
    S.Pc *= S.cn[a] + 2;
  }
  return S;
}

// fine-level fields of the discrete adjoint: ubar (2 x D, ping-pong), the
// predictor-state adjoint (D), fbar (D), Vbar (D), mu0bar (D, also Lbar), mu1bar
// (D*D), the recorded predictor state and flux (2 x D), x of both solves, pbar and
// the adjoint right-hand side
constexpr int kAdjFields(int D) { return 8 * D + D * D + 4; }

// Blocks of the flat PCG passes on a level, or 0 if it does not take them: the
// solver path allows them, 3-D, at least 2^14 cells (smaller levels are launch
// bound and go to the generic kernels or the bottom solve), and rows holding a
// whole number of 16-byte vectors.  (grid: flat_plane_blocks per plane x planes)
constexpr int64_t kFlatMinCells = 1 << 14;
int64_t flat_plane_blocks(const LevelPlan& L, size_t esize) {
  const int64_t W = (int64_t)(16 / esize);
  return (L.n[0] / W * L.n[1] + kFlatThreads - 1) / kFlatThreads;
}
int64_t flat_blocks(const wl_sim_desc& d, const LevelPlan& L, size_t esize) {
  const int W = (int)(16 / esize);
  if (d.ndim != 3 || L.n[0] % W != 0 || (d.solver_path != 0 && d.solver_path != 2)) return 0;
  const int64_t cells = (int64_t)L.n[0] * L.n[1] * L.n[2];
  if (cells < kFlatMinCells) return 0;
  return flat_plane_blocks(L, esize) * L.n[2];
}
// the most flat-pass blocks of any level (they share one partials area)
int64_t flat_blocks_max(const wl_sim_desc& d, const Plan& P) {
  int64_t m = 0;
  for (int l = 0; l < P.nlev; ++l) m = std::max(m, flat_blocks(d, P.lev[l], P.esize));
  return m;
}

Plan make_plan(const wl_sim_desc& d, const std::vector<wl_body_desc>& parts) {
  Plan P;
  P.ndim = d.ndim;
  P.esize = d.prec == WL_F64 ? 8 : 4;
  int n[3] = {(int)d.n[0], (int)d.n[1], d.ndim == 3 ? (int)d.n[2] : 1};
  for (;;) {
    LevelPlan& L = P.lev[P.nlev++];
    for (int a = 0; a < 3; ++a) L.n[a] = n[a];
    const int w = n[0] + 2;
    L.px = ((w + 15) / 16) * 16;  // rows of 64 bytes (FP32) / 128 bytes (FP64)
    L.py = n[1] + 2;
    L.pz = d.ndim == 3 ? n[2] + 2 : 1;
    L.elems = (int64_t)L.px * L.py * L.pz;
    L.alloc = L.elems + 16;
    bool even = true;
    int mn = 1 << 30;
    for (int a = 0; a < d.ndim; ++a) {
      even = even && (n[a] % 2 == 0);
      mn = std::min(mn, n[a] / 2);
    }
    if (!even || mn < 4 || P.nlev == kMaxLevels) break;
    for (int a = 0; a < d.ndim; ++a) n[a] /= 2;
  }
  const int D = d.ndim;
  size_t b = 0;
  const size_t f0 = align256(P.lev[0].alloc * P.esize);
  int nf0 = D /*ua*/ + D /*ub*/ + D /*ft*/ + D /*V*/ + D /*mu0*/ + D * D /*mu1*/ + 1 /*p*/ + 6 /*x r ea eb q iD*/;
  b += nf0 * f0;
  b += align256((size_t)P.lev[0].py * P.lev[0].pz * P.esize);  // exit plane
  for (int l = 1; l < P.nlev; ++l) b += (6 + D) * align256(P.lev[l].alloc * P.esize);
  b += align256((size_t)kNumSlots * kMaxBlocks * sizeof(double));
  b += align256(kNumScal * sizeof(double));
  b += align256(kMaxLevels * sizeof(int));
  {
    const int64_t nf = flat_blocks_max(d, P);  // flat-pass partials and their first stage
    if (nf > 0) b += align256((size_t)(4 * nf + 2 * kFinalizeStage) * sizeof(double));
  }
  if (d.adjoint) b += (size_t)kAdjFields(D) * f0;
  if (d.learned_guess && d.ndim == 3) {
    const PgSizes S = pg_sizes(P);
    b += align256(P.lev[0].alloc * P.esize);  // p_{m-2}
    b += align256(S.Pd * 8) + 2 * align256(S.Pd * 32) + align256(S.Pd * 4);
    b += align256(S.Pc * 8) + 5 * align256(S.Pc * 32) + align256(S.Pc * 4);
    b += kPgRing * (align256(S.Pc * 8) + align256(S.Pc * 4) + align256(S.Pc));
    b += 4 * align256(kPgParams * sizeof(float));
    b += align256(27 * 64 * 2) + 4 * align256(27 * 256 * 2) + 3 * align256(16 * sizeof(float));
    b += align256((size_t)kPgWaves * (27 * 256 + 16) * sizeof(float));
    b += align256(8192 * sizeof(double)) + align256(8 * sizeof(double));
  }
  // sampled parts of the body (FP64): samples, their gradients, the sampled velocity
  for (size_t k = 0; k < parts.size(); ++k)
    if (parts[k].kind == WL_BODY_GRID_SDF) {
      P.grid_cnt[k] = grid_count(parts[k], D);
      P.grid_vel[k] = parts[k].vel_grid != nullptr;
      b += align256(P.grid_cnt[k] * sizeof(double)) + (size_t)D * align256(P.grid_cnt[k] * sizeof(double));
      if (P.grid_vel[k]) b += (size_t)D * align256(P.grid_cnt[k] * sizeof(double));
    }
  P.bytes = b;
  return P;
}

// Map of one part at time t (see wl_body_desc).
void part_motion(const wl_body_desc& b, double t, PartMotion& m) {
  const double w = 2.0 * M_PI * b.freq;
  double eh[3];
  heave_unit(b, eh);
  part_pivot(b, t, m.P);
  const double hd = b.heave_amp * w * std::cos(w * t + b.phase_h);
  for (int k = 0; k < 3; ++k) m.cdot[k] = b.velocity[k] + hd * eh[k];
  const double theta = b.pitch_amp * std::sin(w * t + b.phase_p) + b.spin_omega * t;
  m.ct = std::cos(theta);
  m.st = std::sin(theta);
  m.omega = b.pitch_amp * w * std::cos(w * t + b.phase_p) + b.spin_omega;
  for (int k = 0; k < 3; ++k) {
    m.S[k] = 1.0 + b.scale_amp[k] * std::sin(w * t + b.phase_s);
    m.Sdot[k] = b.scale_amp[k] * w * std::cos(w * t + b.phase_s);
  }
}

void host_motion(const std::vector<wl_body_desc>& ps, double t, Motion& m) {
  m = Motion{};
  for (size_t k = 0; k < ps.size(); ++k) part_motion(ps[k], t, m.m[k]);
}

// ---------------------------------------------------------------------------
// per-kernel timing with HIP events (host objects; enabled on demand)
// ---------------------------------------------------------------------------
struct Profiler {
  static constexpr int kPairs = 1024;
  bool on = false;
  uint32_t groups = ~0u;  // bit k: group k is timed
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<int> kid;
  int cur = -1;
  double ms[WL_K_COUNT] = {};
  int64_t cnt[WL_K_COUNT] = {};

  wl_status enable(hipStream_t s) {
    st = s;
    if (pool.empty()) {
      pool.resize(2 * kPairs);
      for (auto& e : pool)
        if (hipEventCreate(&e) != hipSuccess) return fail(WL_ERR_HIP, "hipEventCreate failed");
    }
    kid.clear();
    for (int k = 0; k < WL_K_COUNT; ++k) {
      ms[k] = 0.0;
      cnt[k] = 0;
    }
    on = true;
    return WL_OK;
  }
  void begin(int k) {
    if (!on || !((groups >> k) & 1u)) return;
    if ((int)kid.size() == kPairs) flush();
    (void)hipEventRecord(pool[2 * kid.size()], st);
    cur = k;
  }
  void end() {
    if (!on || cur < 0) return;
    (void)hipEventRecord(pool[2 * kid.size() + 1], st);
    kid.push_back(cur);
    cur = -1;
  }
  // call only when the stream is idle (after a synchronisation)
  void harvest() {
    for (size_t i = 0; i < kid.size(); ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, pool[2 * i], pool[2 * i + 1]) == hipSuccess) {
        ms[kid[i]] += t;
        cnt[kid[i]] += 1;
      }
    }
    kid.clear();
  }
  void flush() {
    if (kid.empty()) return;
    (void)hipStreamSynchronize(st);
    harvest();
  }
  ~Profiler() {
    for (auto& e : pool) (void)hipEventDestroy(e);
  }
};

#define WL_TIMED(K, LAUNCH) \
  do {                      \
    prof.begin(K);          \
    LAUNCH;                 \
    prof.end();             \
  } while (0)

// ---------------------------------------------------------------------------
// the simulation object
// ---------------------------------------------------------------------------
constexpr int kHostPin = 32;  // doubles of pinned host memory per sim (scalar read-back)

struct SimBase {
  virtual ~SimBase() {}
  virtual wl_status init() = 0;
  virtual wl_status measure(double t) = 0;
  virtual wl_status step(int remeasure, wl_step_stats* st) = 0;
  virtual wl_status apply_bc_cur() = 0;
  virtual wl_status conv_diff() = 0;
  virtual wl_status project_cur(double w, wl_solve_stats* st) = 0;
  virtual wl_status poisson(const void* rhs, void* x, double tol, int itmax, wl_solve_stats* st) = 0;
  virtual wl_status forces(double fp[3], double fv[3]) = 0;
  virtual wl_status forces_static(double* scr, double fp[3], double fv[3]) = 0;
  virtual wl_status field(int which, int level, void** ptr, int64_t shape[4], int64_t strides[4]) = 0;
  virtual wl_status pg_set_weights(const float* w) = 0;
  virtual wl_status pg_get_weights(float* w) = 0;
  virtual wl_status pg_set_mode(int mode, double lr, int iters, int crops, uint64_t seed) = 0;
  virtual wl_status pg_forward(const void* x, const int64_t n[3], float* y) = 0;
  virtual wl_status pg_train(const void* x, const float* t, const unsigned char* m, const int64_t n[3], float* grad,
                             double* loss, int apply) = 0;
  virtual wl_status pg_stats(double* loss, int64_t* steps, int64_t* snaps, int64_t* used, int64_t* tried) = 0;
  virtual wl_status body_update(const wl_body_desc* b) = 0;
  virtual wl_status body_box_of(int level, int lo[3], int hi[3]) = 0;
  virtual wl_status adj_reset() = 0;
  virtual wl_status adj_forces(const double dir[3], double weight, double* value) = 0;
  virtual wl_status adj_step(double tol, wl_step_stats* fst, wl_solve_stats* ast) = 0;
  virtual wl_status adj_step_cfl(double tol, int from_cfl, double* dtbar, wl_step_stats* fst,
                                 wl_solve_stats* ast) = 0;
  virtual wl_status adj_body_grad(double* dR, double* dW) = 0;
  virtual wl_status profile(uint32_t groups) {
    if (groups) {
      prof.groups = groups;
      return prof.enable(stream);
    }
    prof.flush();
    prof.on = false;
    return WL_OK;
  }
  virtual wl_status profile_read(int k, double* ms, int64_t* n) {
    if (k < 0 || k >= WL_K_COUNT) return fail(WL_ERR_INVALID_ARG, "kernel id out of range");
    prof.flush();
    if (ms) *ms = prof.ms[k];
    if (n) *n = prof.cnt[k];
    return WL_OK;
  }
  Profiler prof;
  wl_sim_desc desc;
  std::vector<wl_body_desc> parts;  // the body's parts (next cleared); empty: no body
  Plan plan;
  hipStream_t stream = nullptr;
  double t = 0.0, dt = 0.25;
  double* host_pin = nullptr;  // kHostPin doubles of pinned host memory for read-back
  int device = 0;               // the GPU current at creation
};

template <typename T, int D>
struct Impl : SimBase {
  Grid3 g[kMaxLevels];
  int nb[kMaxLevels];
  int nlev = 1;
  int nb_face = 1;
  BodyP body{};
  bool has_body = false, moving = false;
  T* u[2][3] = {};
  int cur = 0;
  T *ft[3] = {}, *V[3] = {}, *mu0[3] = {}, *mu1[9] = {}, *p = nullptr, *ebuf = nullptr;
  T *x[kMaxLevels] = {}, *r[kMaxLevels] = {}, *e[kMaxLevels][2] = {}, *q[kMaxLevels] = {}, *iD[kMaxLevels] = {};
  T* L[kMaxLevels][3] = {};
  double* red = nullptr;
  double* scal = nullptr;
  int* flags = nullptr;
  Planes planes{};
  int plane_blocks = 1;
  bool exit_valid = false;
  // The coarse part of a multigrid cycle (restriction, the PCG of every coarse
  // level, the bottom solve, prolongation) captured in HIP graphs and replayed:
  // ~150 small launches per cycle, each dispatched faster from a graph (2-3 % of
  // the step on grids of a few million cells).  A graph is reused when the
  // host-side partial counts and the body boxes (launch arguments) are those it
  // was captured with.
  struct VcGraph {
    bool valid = false;
    int pre[kNumSlots] = {}, post[kNumSlots] = {};
    StdBox box[kMaxLevels] = {};
    hipGraphExec_t exec = nullptr;
  };
  static constexpr int kVcGraphs = 4;
  VcGraph vcg[kVcGraphs];
  int vcg_next = 0;
  bool vcg_off = false;  // after a capture that failed: plain launches
  // captures run on a stream of their own (the sim's stream may be the null stream,
  // which cannot be captured); nothing captured executes until the graph is
  // launched on the sim's stream
  hipStream_t cap_stream = nullptr;
  int slot_n[kNumSlots] = {};  // partials written by the last producer of each slot
  int box_lo[3] = {}, box_hi[3] = {};
  bool have_box = false;
  // learned initial guess
  bool pg_on = false, pg_weights_set = false;
  int pg_mode = 0, pg_iters = 1, pg_crops = 2, pg_hist = 0, ring_used = 0, ring_next = 0;
  double pg_lr = 1e-3;
  uint64_t pg_rng = 0;
  int64_t pg_train_steps = 0, pg_snaps = 0, pg_adam_t = 0, pg_used = 0, pg_tried = 0;
  bool pg_loss_pending = false;
  double pg_last_loss = NAN;
  T* p2 = nullptr;
  unsigned short *pgXd = nullptr, *pgA1d = nullptr, *pgA2d = nullptr;
  float* pgYd = nullptr;
  unsigned short *pgXc = nullptr, *pgA1c = nullptr, *pgA2c = nullptr, *pgG3 = nullptr, *pgG2 = nullptr,
                 *pgG1 = nullptr;
  float* pgYc = nullptr;
  unsigned short* ringX[kPgRing] = {};
  float* ringT[kPgRing] = {};
  unsigned char* ringM[kPgRing] = {};
  float *pgW = nullptr, *pgM = nullptr, *pgV = nullptr, *pgGrad = nullptr, *pgPart = nullptr;
  PgWeights pgK{};
  double *pgRed = nullptr, *pgScal = nullptr;
  PgBox bd{}, bcrop{};
  int64_t pgPc = 0;
  int64_t nflat[kMaxLevels] = {};  // blocks of a level's flat PCG passes (0: tiles or generic kernels)
  int64_t wide_n = 0;              // the largest of them
  double* wide = nullptr;          // their partials: sigma, rho_0, rho_{k+1}, max|r| (wide_n
                                   // apart), then 2 x kFinalizeStage first-stage sums
  int tiles[kMaxLevels][4] = {};  // tiled kernels: tiles_x, tiles_y, ntiles (0 = generic kernel), tile depth
  int lbot = 0;                   // first level of the single-workgroup bottom solve
  StdBox sbox[kMaxLevels] = {};   // per level: outside, coefficients are body-free
  // discrete adjoint
  bool adj_on = false, rec = false;
  T* au[2][3] = {};  // ubar ping-pong; au[acur] is the adjoint of the current state
  int acur = 0;
  T *aup[3] = {}, *afb[3] = {}, *aVb[3] = {}, *am0b[3] = {}, *am1b[9] = {}, *recB[3] = {}, *recF[3] = {};
  T *recX1 = nullptr, *recX2 = nullptr, *apb = nullptr, *arhs = nullptr;
  // FP64 copies of the sampled parts: samples, gradients (D arrays), velocity (D arrays)
  double *gsd[kMaxParts] = {}, *ggr[kMaxParts] = {}, *gvl[kMaxParts] = {};
  double adj_dR = 0.0;  // direct radius derivative of the force functionals so far

  Vec3<T> v3(T* const a[3]) const {
    Vec3<T> v;
    for (int k = 0; k < 3; ++k) v.c[k] = a[k];
    return v;
  }
  Vec9<T> v9(T* const a[9]) const {
    Vec9<T> v;
    for (int k = 0; k < 9; ++k) v.c[k] = a[k];
    return v;
  }
  double* slot(int s) const { return red + (size_t)s * kMaxBlocks; }
  // whole-allocation copy of a fine-level field (front padding included)
  hipError_t copy_field(T* dst, const T* src) {
    return hipMemcpyAsync(dst - kFrontPad, src - kFrontPad, plan.lev[0].alloc * sizeof(T), hipMemcpyDeviceToDevice,
                          stream);
  }
  void fill_field(T* a, T v) {
    k_fill<T><<<blocks_for(plan.lev[0].alloc), kBlock, 0, stream>>>(a - kFrontPad, plan.lev[0].alloc, v);
  }

  // Assign every field an offset in the workspace; returns the bytes used.
  size_t carve(char* base) {
    nlev = plan.nlev;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      char* p_ = base + off;
      off += align256(bytes);
      return p_;
    };
    // a field starts kFrontPad elements into its allocation: interior rows are then
    // 64-byte aligned and the flat kernels sweep the whole aligned allocation
    auto field = [&](int l) { return (T*)take(plan.lev[l].alloc * sizeof(T)) + kFrontPad; };
    for (int k = 0; k < D; ++k) u[0][k] = field(0);
    for (int k = 0; k < D; ++k) u[1][k] = field(0);
    for (int k = 0; k < D; ++k) ft[k] = field(0);
    for (int k = 0; k < D; ++k) V[k] = field(0);
    for (int k = 0; k < D; ++k) mu0[k] = field(0);
    for (int k = 0; k < D * D; ++k) mu1[k] = field(0);
    p = field(0);
    x[0] = field(0);
    r[0] = field(0);
    e[0][0] = field(0);
    e[0][1] = field(0);
    q[0] = field(0);
    iD[0] = field(0);
    for (int k = 0; k < D; ++k) L[0][k] = mu0[k];
    ebuf = (T*)take((size_t)plan.lev[0].py * plan.lev[0].pz * sizeof(T));
    for (int l = 1; l < nlev; ++l) {
      x[l] = field(l);
      r[l] = field(l);
      e[l][0] = field(l);
      e[l][1] = field(l);
      q[l] = field(l);
      iD[l] = field(l);
      for (int k = 0; k < D; ++k) L[l][k] = field(l);
    }
    red = (double*)take((size_t)kNumSlots * kMaxBlocks * sizeof(double));
    scal = (double*)take(kNumScal * sizeof(double));
    flags = (int*)take(kMaxLevels * sizeof(int));
    wide_n = flat_blocks_max(desc, plan);
    for (int l = 0; l < plan.nlev; ++l) nflat[l] = flat_blocks(desc, plan.lev[l], sizeof(T));
    if (wide_n > 0) wide = (double*)take((size_t)(4 * wide_n + 2 * kFinalizeStage) * sizeof(double));
    adj_on = desc.adjoint != 0;
    if (adj_on) {
      for (int k = 0; k < D; ++k) au[0][k] = field(0);
      for (int k = 0; k < D; ++k) au[1][k] = field(0);
      for (int k = 0; k < D; ++k) aup[k] = field(0);
      for (int k = 0; k < D; ++k) afb[k] = field(0);
      for (int k = 0; k < D; ++k) aVb[k] = field(0);
      for (int k = 0; k < D; ++k) am0b[k] = field(0);
      for (int k = 0; k < D * D; ++k) am1b[k] = field(0);
      for (int k = 0; k < D; ++k) recB[k] = field(0);
      for (int k = 0; k < D; ++k) recF[k] = field(0);
      recX1 = field(0);
      recX2 = field(0);
      apb = field(0);
      arhs = field(0);
    }
    pg_on = desc.learned_guess && D == 3;
    if (pg_on) {
      const PgSizes S = pg_sizes(plan);
      p2 = field(0);
      pgXd = (unsigned short*)take(S.Pd * 8);
      pgA1d = (unsigned short*)take(S.Pd * 32);
      pgA2d = (unsigned short*)take(S.Pd * 32);
      pgYd = (float*)take(S.Pd * 4);
      pgXc = (unsigned short*)take(S.Pc * 8);
      pgA1c = (unsigned short*)take(S.Pc * 32);
      pgA2c = (unsigned short*)take(S.Pc * 32);
      pgG3 = (unsigned short*)take(S.Pc * 32);
      pgG2 = (unsigned short*)take(S.Pc * 32);
      pgG1 = (unsigned short*)take(S.Pc * 32);
      pgYc = (float*)take(S.Pc * 4);
      for (int k = 0; k < kPgRing; ++k) {
        ringX[k] = (unsigned short*)take(S.Pc * 8);
        ringT[k] = (float*)take(S.Pc * 4);
        ringM[k] = (unsigned char*)take(S.Pc);
      }
      pgW = (float*)take(kPgParams * sizeof(float));
      pgM = (float*)take(kPgParams * sizeof(float));
      pgV = (float*)take(kPgParams * sizeof(float));
      pgGrad = (float*)take(kPgParams * sizeof(float));
      pgK.w1f = (unsigned short*)take(27 * 64 * 2);
      pgK.w2f = (unsigned short*)take(27 * 256 * 2);
      pgK.w3f = (unsigned short*)take(27 * 256 * 2);
      pgK.w3b = (unsigned short*)take(27 * 256 * 2);
      pgK.w2b = (unsigned short*)take(27 * 256 * 2);
      pgK.b1 = (float*)take(16 * sizeof(float));
      pgK.b2 = (float*)take(16 * sizeof(float));
      pgK.b3 = (float*)take(16 * sizeof(float));
      pgPart = (float*)take((size_t)kPgWaves * (27 * 256 + 16) * sizeof(float));
      pgRed = (double*)take(8192 * sizeof(double));
      pgScal = (double*)take(8 * sizeof(double));
      for (int a = 0; a < 3; ++a) {
        bd.n[a] = plan.lev[0].n[a];
        bd.P[a] = bd.n[a] + 2;
        bcrop.n[a] = S.cn[a];
        bcrop.P[a] = bcrop.n[a] + 2;
      }
      pgPc = S.Pc;
    }
    for (int k = 0; k < kMaxParts; ++k) {
      gsd[k] = ggr[k] = gvl[k] = nullptr;
      if (plan.grid_cnt[k] == 0) continue;
      const size_t gb = plan.grid_cnt[k] * sizeof(double);
      gsd[k] = (double*)take(gb);
      ggr[k] = (double*)take(D * align256(gb));
      if (plan.grid_vel[k]) gvl[k] = (double*)take(D * align256(gb));
    }
    return off;
  }

  // every buffer a kernel may touch is carved (non-NULL) and inside [base, base + bytes)
  bool carved_ok(const char* base, size_t bytes) const {
    auto in = [&](const void* q) { return q && (const char*)q >= base && (const char*)q < base + bytes; };
    bool ok = in(p) && in(ebuf) && in(red) && in(scal) && in(flags);
    for (int k = 0; k < D; ++k) ok = ok && in(u[0][k]) && in(u[1][k]) && in(ft[k]) && in(V[k]) && in(mu0[k]);
    for (int k = 0; k < D * D; ++k) ok = ok && in(mu1[k]);
    if (adj_on) {
      ok = ok && in(recX1) && in(recX2) && in(apb) && in(arhs);
      for (int k = 0; k < D; ++k)
        ok = ok && in(au[0][k]) && in(au[1][k]) && in(aup[k]) && in(afb[k]) && in(aVb[k]) && in(am0b[k]) &&
             in(recB[k]) && in(recF[k]);
      for (int k = 0; k < D * D; ++k) ok = ok && in(am1b[k]);
      ok = ok && (const char*)(arhs - kFrontPad + plan.lev[0].alloc) <= base + bytes;
    }
    for (int l = 0; l < nlev; ++l) {
      ok = ok && in(x[l]) && in(r[l]) && in(e[l][0]) && in(e[l][1]) && in(q[l]) && in(iD[l]);
      for (int k = 0; k < D; ++k) ok = ok && in(L[l][k]);
    }
    if (pg_on) {
      ok = ok && in(p2) && in(pgXd) && in(pgA1d) && in(pgA2d) && in(pgYd) && in(pgXc) && in(pgA1c) && in(pgA2c) &&
           in(pgG3) && in(pgG2) && in(pgG1) && in(pgYc) && in(pgW) && in(pgM) && in(pgV) && in(pgGrad) &&
           in(pgK.w1f) && in(pgK.w2f) && in(pgK.w3f) && in(pgK.w3b) && in(pgK.w2b) && in(pgK.b1) && in(pgK.b2) &&
           in(pgK.b3) && in(pgPart) && in(pgRed) && in(pgScal);
      for (int k = 0; k < kPgRing; ++k) ok = ok && in(ringX[k]) && in(ringT[k]) && in(ringM[k]);
      // the last byte of the last buffer must be inside the workspace too
      ok = ok && (const char*)(pgScal + 8) <= base + bytes;
    }
    for (int k = 0; k < kMaxParts; ++k) {
      const int64_t c = plan.grid_cnt[k];
      if (c == 0) continue;
      ok = ok && in(gsd[k]) && in(ggr[k]) && (const char*)(ggr[k] + D * c) <= base + bytes;
      if (plan.grid_vel[k]) ok = ok && in(gvl[k]) && (const char*)(gvl[k] + D * c) <= base + bytes;
    }
    return ok;
  }

  void setup_grids() {
    nlev = plan.nlev;
    for (int l = 0; l < nlev; ++l) {
      const LevelPlan& P = plan.lev[l];
      for (int a = 0; a < 3; ++a) {
        g[l].n[a] = P.n[a];
        g[l].per[a] = (a < D) ? ((desc.periodic_mask >> a) & 1u) : 0;
      }
      g[l].s[0] = 1;
      g[l].s[1] = P.px;
      g[l].s[2] = P.px * P.py;
      nb[l] = blocks_for((int64_t)P.n[0] * P.n[1] * (D == 3 ? P.n[2] : 1));
      tiles[l][0] = tiles[l][1] = tiles[l][2] = tiles[l][3] = 0;
      if (D == 3 && desc.solver_path != 3 && P.n[0] >= 32 && P.n[1] >= 8 &&
          (int64_t)P.n[0] * P.n[1] * P.n[2] >= (1 << 18)) {
        const int tx = (P.n[0] + kTX - 1) / kTX, ty = (P.n[1] + kTY - 1) / kTY;
        // march depth: kTZ planes, shortened on the smaller levels until there
        // are about four tiles per compute unit (a march shorter than
        // kTileMinZ planes would spend most of its loads on the pipeline fill)
        int depth = kTZ;
        while (depth > kTileMinZ && (int64_t)tx * ty * ((P.n[2] + depth - 1) / depth) < kTileTarget) depth /= 2;
        const int tz = (P.n[2] + depth - 1) / depth;
        if ((int64_t)tx * ty * tz <= kMaxBlocks) {
          tiles[l][0] = tx;
          tiles[l][1] = ty;
          tiles[l][2] = tx * ty * tz;
          tiles[l][3] = depth;
        }
      }
    }
    nb_face = blocks_for((int64_t)(g[0].n[0] + 2) * (g[0].n[1] + 2) * (D == 3 ? g[0].n[2] + 2 : 1));
    planes.count = 0;
    int maxarea = 1;
    for (int c = 0; c < D; ++c)
      for (int a = 0; a < D; ++a) {
        const int N = g[0].n[a];
        int ids[3] = {0, N + 1, 1};
        const int cnt = (a == c && !g[0].per[a]) ? 3 : 2;
        for (int k = 0; k < cnt; ++k) planes.p[planes.count++] = Plane{c, a, ids[k]};
        int area = 1;
        for (int o = 0; o < D; ++o)
          if (o != a) area *= g[0].n[o] + 2;
        maxarea = std::max(maxarea, area);
      }
    plane_blocks = blocks_for(maxarea);
    lbot = bottom_level();
  }

  // Device description of the body from its parts; the sampled parts point at
  // their FP64 copies in the workspace.
  void build_body() {
    body = BodyP{};
    has_body = !parts.empty();
    body.nparts = (int)parts.size();
    body.general = parts_general(parts) ? 1 : 0;
    moving = false;
    for (size_t k = 0; k < parts.size(); ++k) {
      const wl_body_desc& b = parts[k];
      PartP& q = body.p[k];
      q.kind = b.kind;
      q.op = k == 0 ? kOpUnion : b.op;
      q.R = b.radius;
      q.shell = b.shell;
      double nm = 0;
      for (int a = 0; a < D; ++a) nm += b.normal[a] * b.normal[a];
      nm = std::sqrt(nm);
      for (int a = 0; a < 3; ++a) {
        q.h[a] = b.half_extent[a];
        q.po[a] = b.pivot_offset[a];
        q.nrm[a] = (a < D && nm > 0.0) ? b.normal[a] / nm : 0.0;
      }
      if (b.kind == WL_BODY_GRID_SDF) {
        q.gs.s = gsd[k];
        q.gs.gr = ggr[k];
        q.gs.v = plan.grid_vel[k] ? gvl[k] : nullptr;
        for (int a = 0; a < 3; ++a) {
          q.gs.n[a] = a < D ? (int)b.grid_n[a] : 1;
          q.gs.o[a] = a < D ? b.grid_origin[a] : 0.0;
        }
        q.gs.h = b.grid_h;
      }
      moving = moving || part_moving(b);
    }
  }

  // FP64 copies of the sampled parts and their gradients (read from the caller's arrays)
  wl_status upload_grids() {
    for (size_t k = 0; k < parts.size(); ++k) {
      const wl_body_desc& b = parts[k];
      if (b.kind != WL_BODY_GRID_SDF) continue;
      const int64_t cnt = plan.grid_cnt[k];
      k_widen<T><<<blocks_for(cnt), kBlock, 0, stream>>>((const T*)b.sdf_grid, gsd[k], cnt);
      k_grid_grad<D><<<blocks_for(cnt), kBlock, 0, stream>>>(gsd[k], ggr[k], (int)b.grid_n[0], (int)b.grid_n[1],
                                                              D == 3 ? (int)b.grid_n[2] : 1, b.grid_h);
      if (plan.grid_vel[k])
        k_widen<T><<<blocks_for(D * cnt), kBlock, 0, stream>>>((const T*)b.vel_grid, gvl[k], D * cnt);
    }
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  wl_status init() override {
    build_body();
    setup_grids();
    {
      wl_status s0 = upload_grids();
      if (s0 != WL_OK) return s0;
    }
    for (int c = 0; c < D; ++c) {
      k_fill<T><<<blocks_for(plan.lev[0].elems), kBlock, 0, stream>>>(u[cur][c], plan.lev[0].elems, T(desc.U[c]));
      k_fill<T><<<blocks_for(plan.lev[0].elems), kBlock, 0, stream>>>(u[1 - cur][c], plan.lev[0].elems, T(desc.U[c]));
    }
    WL_HIP(hipGetLastError());
    t = 0.0;
    dt = desc.dt0;
    return measure(0.0);
  }

  // Inverse diagonals and coarse coefficients after the faces lo..hi (padded
  // indices, inclusive) of the fine level were re-measured: on every level only
  // the faces that depend on them and the cells next to those faces.
  wl_status coefficients(const int lo[3], const int hi[3]) {
    int flo[3], fhi[3];  // changed faces of the current level
    for (int a = 0; a < 3; ++a) {
      flo[a] = a < D ? lo[a] : 0;
      fhi[a] = a < D ? hi[a] : 0;
    }
    for (int l = 0; l < nlev; ++l) {
      if (l > 0) {
        // coarse face J takes the fine faces 2J-1 (its own axis) and 2J-1, 2J (the others)
        int clo[3], chi[3], m = 1;
        for (int a = 0; a < 3; ++a) {
          clo[a] = a < D ? std::max(1, flo[a] / 2) : 0;
          chi[a] = a < D ? std::min(g[l].n[a] + 1, (fhi[a] + 2) / 2) : 0;
          if (a < D) m *= std::max(0, chi[a] - clo[a] + 1);
        }
        if (m > 0)
          WL_TIMED(WL_K_COEF, (k_restrict_L<T, D><<<dim3(blocks_for(m), D), kBlock, 0, stream>>>(
                                  g[l - 1], g[l], v3(L[l - 1]), v3(L[l]), make_int3(clo[0], clo[1], clo[2]),
                                  make_int3(chi[0], chi[1], chi[2]))));
        for (int a = 0; a < 3; ++a) {
          flo[a] = clo[a];
          fhi[a] = chi[a];
        }
      }
      // cells whose faces (I, I+1 along each axis) changed; a periodic axis whose
      // changed range reaches its ends is taken whole (the wrapped face)
      int cl[3], ch[3];
      int64_t m = 1;
      for (int a = 0; a < 3; ++a) {
        if (a >= D) {
          cl[a] = ch[a] = 0;
          continue;
        }
        cl[a] = std::max(1, flo[a] - 1);
        ch[a] = std::min(g[l].n[a], fhi[a]);
        if (g[l].per[a] && (flo[a] <= 1 || fhi[a] >= g[l].n[a])) {
          cl[a] = 1;
          ch[a] = g[l].n[a];
        }
        m *= std::max(0, ch[a] - cl[a] + 1);
      }
      if (m > 0)
        WL_TIMED(WL_K_COEF, (k_inv_diag<T, D><<<blocks_for(m), kBlock, 0, stream>>>(
                                g[l], v3(L[l]), iD[l], make_int3(cl[0], cl[1], cl[2]), make_int3(ch[0], ch[1], ch[2]))));
    }
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  // Index box (padded coordinates) outside of which measure leaves mu0 = 1 (0 on
  // boundary faces), mu1 = 0, V = 0 at time tm: the body's extent (every point
  // where d < 2 + eps can hold) with a 3-cell margin.  Empty: lo = 1, hi = 0.
  void body_box(double tm, int lo[3], int hi[3]) const {
    double wlo[3], whi[3];
    body_extent(parts, D, desc.eps, tm, false, 3.0, wlo, whi);
    bool empty = false;
    for (int a = 0; a < 3; ++a) {
      if (a >= D) {
        lo[a] = hi[a] = 0;
        continue;
      }
      lo[a] = std::isinf(wlo[a]) ? 0 : (int)std::max(0.0, std::floor(wlo[a]));
      hi[a] = std::isinf(whi[a]) ? g[0].n[a] + 1 : (int)std::min(double(g[0].n[a] + 1), std::ceil(whi[a]) + 2.0);
      if (wlo[a] > whi[a] || lo[a] > hi[a]) empty = true;
    }
    if (empty)
      for (int a = 0; a < 3; ++a) {
        lo[a] = 1;
        hi[a] = 0;
      }
  }

  // Body boxes of every level from the fine one (box_lo/hi, or empty without a body).
  // Coarse face/cell J covers fine indices 2J-1 and 2J, so J outside
  // [floor(lo/2) - 1, floor((hi+1)/2) + 1] has all its fine indices outside [lo, hi].
  void update_sbox() {
    int lo[3] = {1, 1, 1}, hi[3] = {0, 0, 0};
    if (has_body && have_box)
      for (int a = 0; a < 3; ++a) {
        lo[a] = a < D ? box_lo[a] : 0;
        hi[a] = a < D ? box_hi[a] : 0;
      }
    double Ls = 1.0;
    for (int l = 0; l < nlev; ++l) {
      for (int a = 0; a < 3; ++a) {
        sbox[l].lo[a] = lo[a];
        sbox[l].hi[a] = hi[a];
      }
      sbox[l].Lstd = Ls;
      for (int c = 0; c < 4; ++c) {
        sbox[l].iDf[c] = 1.0f / (-((float)Ls * (float)(2 * D - c)));
        sbox[l].iDd[c] = 1.0 / (-(Ls * (double)(2 * D - c)));
      }
      if (lo[0] <= hi[0])
        for (int a = 0; a < D; ++a) {
          lo[a] = std::max(0, lo[a] / 2 - 1);
          hi[a] = std::min(g[l + 1 < nlev ? l + 1 : l].n[a] + 1, (hi[a] + 1) / 2 + 1);
        }
      Ls *= (D == 3) ? 2.0 : 1.0;
    }
  }

  wl_status measure_box(double tm, const int lo[3], const int hi[3]) {
    Motion m{};
    if (has_body) host_motion(parts, tm, m);
    int64_t vol = 1;
    for (int a = 0; a < D; ++a) vol *= std::max(0, hi[a] - lo[a] + 1);
    if (vol == 0) return WL_OK;
    const int3 l3 = make_int3(lo[0], lo[1], lo[2]), h3 = make_int3(hi[0], hi[1], hi[2]);
    WL_TIMED(WL_K_MEASURE, (k_measure<T, D><<<dim3(blocks_for(vol), D), kBlock, 0, stream>>>(
                               g[0], body, m, desc.eps, v3(mu0), v9(mu1), v3(V), l3, h3)));
    WL_HIP(hipGetLastError());
    return coefficients(lo, hi);
  }

  // full-domain measure (creation and explicit calls)
  wl_status measure(double tm) override {
    int lo[3] = {0, 0, 0}, hi[3] = {g[0].n[0] + 1, g[0].n[1] + 1, D == 3 ? g[0].n[2] + 1 : 0};
    wl_status s = measure_box(tm, lo, hi);
    if (s == WL_OK && has_body) {
      body_box(tm, box_lo, box_hi);
      have_box = true;
    }
    update_sbox();
    return s;
  }

  // per-step re-measure of a moving body: only the union of the previous and the
  // current body boxes can change
  wl_status remeasure_moving(double tm) {
    // a translating body must not reach the non-periodic faces
    wl_status s = check_reach(desc, parts, tm, false);
    if (s != WL_OK) return s;
    if (!have_box) return measure(tm);
    int lo[3], hi[3];
    body_box(tm, lo, hi);
    int ul[3], uh[3];
    const bool new_empty = lo[0] > hi[0], old_empty = box_lo[0] > box_hi[0];
    for (int a = 0; a < 3; ++a) {
      ul[a] = new_empty ? box_lo[a] : (old_empty ? lo[a] : std::min(lo[a], box_lo[a]));
      uh[a] = new_empty ? box_hi[a] : (old_empty ? hi[a] : std::max(hi[a], box_hi[a]));
    }
    s = measure_box(tm, ul, uh);
    for (int a = 0; a < 3; ++a) {
      box_lo[a] = lo[a];
      box_hi[a] = hi[a];
    }
    update_sbox();
    return s;
  }

  wl_status bc(T* const uu[3], bool use_exit) {
    WL_TIMED(WL_K_BC, (k_bc<T, D><<<dim3(plane_blocks, planes.count), kBlock, 0, stream>>>(
                          g[0], v3(uu), planes, desc.U[0], desc.U[1], desc.U[2], ebuf, scal, use_exit ? 1 : 0)));
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  wl_status apply_bc_cur() override { return bc(u[cur], false); }

  wl_status read_scalar_max(int s, double* out) {
    WL_TIMED(WL_K_REDUCE, (k_finalize_max<<<1, kBlock, 0, stream>>>(slot(s), slot_n[s], scal + kScalRmax)));
    WL_HIP(hipGetLastError());
    WL_HIP(hipMemcpyAsync(host_pin, scal + kScalRmax, sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    prof.harvest();
    *out = host_pin[0];
    return WL_OK;
  }

  void set_mean_producer(int grid) { slot_n[kSlotSumR] = slot_n[kSlotCnt] = grid; }
  // flat BDIM blend: the vectors of the padded rows of a plane x the padded planes x D
  // k_bdim_flat: the row vectors of x-faces 1..N, then the two x ghost faces of
  // every row, of each padded plane and component
  dim3 bdim_grid() const {
    const int vr2 = g[0].n[0] / Vec16<T>::W + 2;
    return dim3((unsigned)((vr2 * (g[0].n[1] + 2) + kFlatThreads - 1) / kFlatThreads), (unsigned)(g[0].n[2] + 2),
                (unsigned)D);
  }
  dim3 flat_grid(int l) const {
    return dim3((unsigned)flat_plane_blocks(plan.lev[l], sizeof(T)), (unsigned)g[l].n[2]);
  }

  // Sum (or max) a slot's partials into its first entry when a large grid left
  // them: each block of the consumer would otherwise re-add all of them.
  static constexpr int kCollapseMin = 2048;
  // A flat launch leaves its partials in the slots for the consumers to add only
  // up to this many blocks, else they are totalled first (256 against 2048 saves
  // ~0.15 % of the plate step: one finalize launch costs less than every block of
  // a 1728-block level re-adding the partials).
  static constexpr int kFlatDirectMax = 256;
  // Totals of n partials into slot sa / sb (sb < 0: none): in two stages when
  // there are many (a single block would wait on each load in turn).
  void reduce_wide(const double* a, int a_max, const double* b, int b_max, int n, int sa, int sb) {
    double* out_b = sb >= 0 ? slot(sb) : nullptr;
    if (n > 16 * kFinalizeThreads || desc.reduce_mode == 2) {
      double* ta = wide + 4 * wide_n;
      double* tb = ta + kFinalizeStage;
      WL_TIMED(WL_K_REDUCE, (k_finalize2<<<kFinalizeStage, kFinalizeThreads, 0, stream>>>(
                                a, a_max, sb >= 0 ? b : nullptr, b_max, n, ta, tb)));
      WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(ta, a_max, sb >= 0 ? tb : nullptr, b_max,
                                                                             kFinalizeStage, slot(sa), out_b)));
    } else {
      WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(a, a_max, sb >= 0 ? b : nullptr, b_max, n,
                                                                             slot(sa), out_b)));
    }
    slot_n[sa] = 1;
    if (sb >= 0) slot_n[sb] = 1;
  }

  void collapse(int sa, int a_max, int sb, int b_max) {
    const int n = slot_n[sa];
    if (n <= kCollapseMin) return;
    WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(
                              slot(sa), a_max, sb >= 0 ? slot(sb) : nullptr, b_max, n, slot(sa),
                              sb >= 0 ? slot(sb) : nullptr)));
    slot_n[sa] = 1;
    if (sb >= 0) slot_n[sb] = 1;
  }

  void pcg(int l, bool fine) {
    const int K = desc.pcg_iters;
    T* eo = e[l][0];
    T* en = e[l][1];
    const int64_t nvec = plan.lev[l].alloc / Vec16<T>::W;
    const int gb = blocks_for(nvec);
    const int kidA = l == 0 ? WL_K_PCG_A : WL_K_COARSE, kidB = l == 0 ? WL_K_PCG_B : WL_K_COARSE;
    const int nf = (int)nflat[l];
    // a flat level with few blocks leaves its partials in the slots, as the tiles do
    const bool direct = nf > 0 && nf <= kFlatDirectMax && desc.reduce_mode == 0;
    collapse(kSlotSumR, 0, kSlotCnt, 0);
    for (int k = 0; k < K; ++k) {
      const int wr = k < K - 1 ? 1 : 0, wm = (fine && k == K - 1) ? 1 : 0;
      RedN rn{slot_n[kSlotSumR], slot_n[kSlotRho0 + k], k > 0 ? slot_n[kSlotRho0 + k - 1] : 0, 0};
      int ga;
      double* const wsig = direct ? slot(kSlotSig0 + k) : wide;
      double* const wrho0 = direct ? slot(kSlotRho0) : wide + wide_n;
      double* const wrho = direct ? slot(kSlotRho0 + k + 1) : wide + 2 * wide_n;
      double* const wmax = direct ? slot(kSlotRmax) : wide + 3 * wide_n;
      if (nf > 0) {
        if (desc.periodic_mask) {
          if (l == 0)
            WL_TIMED(kidA, (k_pcg_a_fused_flat<T, true, 1><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                g[l], v3(L[l]), iD[l], r[l], eo, en, red, k, rn, wsig, wrho0, flags + l, sbox[l])));
          else
            WL_TIMED(kidA, (k_pcg_a_fused_flat<T, true, 0><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                g[l], v3(L[l]), iD[l], r[l], eo, en, red, k, rn, wsig, wrho0, flags + l, sbox[l])));
        } else {
          if (l == 0)
            WL_TIMED(kidA, (k_pcg_a_fused_flat<T, false, 1><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                g[l], v3(L[l]), iD[l], r[l], eo, en, red, k, rn, wsig, wrho0, flags + l, sbox[l])));
          else
            WL_TIMED(kidA, (k_pcg_a_fused_flat<T, false, 0><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                g[l], v3(L[l]), iD[l], r[l], eo, en, red, k, rn, wsig, wrho0, flags + l, sbox[l])));
        }
        ga = 1;
      } else if (tiles[l][2] > 0) {
        ga = tiles[l][2];
        // q is not stored: the tiled pass B recomputes it
        if (l == 0)
          WL_TIMED(kidA, (k_pcg_a_tile<T, 1, 0><<<ga, kTileThreads, 0, stream>>>(
                              g[l], v3(L[l]), iD[l], r[l], eo, en, q[l], red, k, rn, slot(kSlotSig0 + k),
                              flags + l, tiles[l][0], tiles[l][1], tiles[l][2], tiles[l][3], sbox[l])));
        else
          WL_TIMED(kidA, (k_pcg_a_tile<T, 0, 0><<<ga, kTileThreads, 0, stream>>>(
                              g[l], v3(L[l]), iD[l], r[l], eo, en, q[l], red, k, rn, slot(kSlotSig0 + k),
                              flags + l, tiles[l][0], tiles[l][1], tiles[l][2], tiles[l][3], sbox[l])));
      } else {
        ga = nb[l];
        if (l == 0)
          WL_TIMED(kidA, (k_pcg_a<T, D, 1><<<ga, kBlock, 0, stream>>>(g[l], v3(L[l]), iD[l], r[l], eo, en, q[l],
                                                                      red, k, rn, slot(kSlotSig0 + k), flags + l)));
        else
          WL_TIMED(kidA, (k_pcg_a<T, D, 0><<<ga, kBlock, 0, stream>>>(g[l], v3(L[l]), iD[l], r[l], eo, en, q[l],
                                                                      red, k, rn, slot(kSlotSig0 + k), flags + l)));
      }
      if (nf > 0 && !direct) {
        reduce_wide(wsig, 0, wrho0, 0, nf, kSlotSig0 + k, k == 0 ? kSlotRho0 : -1);
      } else if (nf > 0) {
        slot_n[kSlotSig0 + k] = nf;
        if (k == 0) slot_n[kSlotRho0] = nf;
      } else {
        slot_n[kSlotSig0 + k] = ga;
        if (k == 0) slot_n[kSlotRho0] = ga;
        collapse(kSlotSig0 + k, 0, k == 0 ? kSlotRho0 : -1, 0);
      }
      rn.sig = slot_n[kSlotSig0 + k];
      rn.rho = slot_n[kSlotRho0 + k];
      T* b_iD = iD[l] - kFrontPad;
      T* b_e = en - kFrontPad;
      T* b_q = q[l] - kFrontPad;
      T* b_x = x[l] - kFrontPad;
      T* b_r = r[l] - kFrontPad;
      int gbk = gb;
      if (nf > 0) {
        if (desc.periodic_mask)
          {
            if (l == 0)
              WL_TIMED(kidB, (k_pcg_b_flat<T, true, 1><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                  g[l], v3(L[l]), iD[l], en, x[l], r[l], red, k, rn, wrho, wmax, wr, wm, flags + l,
                                  sbox[l])));
            else
              WL_TIMED(kidB, (k_pcg_b_flat<T, true, 0><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                  g[l], v3(L[l]), iD[l], en, x[l], r[l], red, k, rn, wrho, wmax, wr, wm, flags + l,
                                  sbox[l])));
          }
        else
          {
            if (l == 0)
              WL_TIMED(kidB, (k_pcg_b_flat<T, false, 1><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                  g[l], v3(L[l]), iD[l], en, x[l], r[l], red, k, rn, wrho, wmax, wr, wm, flags + l,
                                  sbox[l])));
            else
              WL_TIMED(kidB, (k_pcg_b_flat<T, false, 0><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                                  g[l], v3(L[l]), iD[l], en, x[l], r[l], red, k, rn, wrho, wmax, wr, wm, flags + l,
                                  sbox[l])));
          }
        if (direct) {
          if (wr) slot_n[kSlotRho0 + k + 1] = nf;
          if (wm) slot_n[kSlotRmax] = nf;
        } else if (wr) {
          reduce_wide(wrho, 0, wmax, 1, nf, kSlotRho0 + k + 1, wm ? kSlotRmax : -1);
        } else if (wm) {
          reduce_wide(wmax, 1, nullptr, 0, nf, kSlotRmax, -1);
        }
        gbk = 1;
      } else if (tiles[l][2] > 0) {
        gbk = tiles[l][2];
        if (l == 0)
          WL_TIMED(kidB, (k_pcg_b_tile<T, 1><<<gbk, kTileThreads, 0, stream>>>(
                              g[l], v3(L[l]), iD[l], en, x[l], r[l], red, k, rn, slot(kSlotRho0 + k + 1),
                              slot(kSlotRmax), wr, wm, flags + l, tiles[l][0], tiles[l][1], tiles[l][2], tiles[l][3], sbox[l])));
        else
          WL_TIMED(kidB, (k_pcg_b_tile<T, 0><<<gbk, kTileThreads, 0, stream>>>(
                              g[l], v3(L[l]), iD[l], en, x[l], r[l], red, k, rn, slot(kSlotRho0 + k + 1),
                              slot(kSlotRmax), wr, wm, flags + l, tiles[l][0], tiles[l][1], tiles[l][2], tiles[l][3], sbox[l])));
      } else if (l == 0) {
        WL_TIMED(kidB, (k_pcg_b<T, D, 1><<<gb, kBlock, 0, stream>>>(nvec, b_iD, b_e, b_q, b_x, b_r, red, k, rn,
                                                                    slot(kSlotRho0 + k + 1), slot(kSlotRmax), wr,
                                                                    wm, flags + l, g[l], sbox[l])));
      } else {
        WL_TIMED(kidB, (k_pcg_b<T, D, 0><<<gb, kBlock, 0, stream>>>(nvec, b_iD, b_e, b_q, b_x, b_r, red, k, rn,
                                                                    slot(kSlotRho0 + k + 1), slot(kSlotRmax), wr,
                                                                    wm, flags + l, g[l], sbox[l])));
      }
      if (nf == 0) {
        if (wr) slot_n[kSlotRho0 + k + 1] = gbk;
        if (wm) slot_n[kSlotRmax] = gbk;
        if (wr)
          collapse(kSlotRho0 + k + 1, 0, wm ? kSlotRmax : -1, 1);
        else if (wm)
          collapse(kSlotRmax, 1, -1, 0);
      }
      std::swap(eo, en);
    }
  }

  // first level of the single-workgroup bottom solve (nlev if none): the first
  // coarse level with at most kBottomCells cells, if the levels below fit
  int bottom_level() const {
    for (int l = 1; l < nlev; ++l) {
      int64_t cells = 1, padded = 1;
      for (int a = 0; a < D; ++a) {
        cells *= g[l].n[a];
        padded *= g[l].n[a] + 2;
      }
      // the coarser levels are smaller still, so the first one decides
      if (cells <= kBottomCells && padded <= bottom_lds_elems<T>()) return (nlev - l <= kBottomMax) ? l : nlev;
    }
    return nlev;
  }

  void bottom(int lb) {
    BottomLevels<T> bl{};
    bl.n = nlev - lb;
    bl.pcg_iters = desc.pcg_iters;
    for (int l = lb; l < nlev; ++l) {
      LevelRef<T>& v = bl.lv[l - lb];
      v.g = g[l];
      v.x = x[l];
      v.r = r[l];
      v.e = e[l][0];
      v.q = q[l];
      v.iD = iD[l];
      v.L = v3(L[l]);
    }
    WL_TIMED(WL_K_COARSE, (k_bottom<T, D><<<1, kBottom, 0, stream>>>(bl)));
  }

  bool vcg_allowed() const {
    if (vcg_off || desc.vcycle_graph == 1) return false;
    // a moving body changes the body boxes (launch arguments) as it goes, and each
    // new box costs a capture: automatic mode keeps plain launches for it
    if (desc.vcycle_graph == 0 && moving) return false;
    // events cannot be recorded inside a graph: no graph while its kernels are timed
    constexpr uint32_t inside =
        (1u << WL_K_RESTRICT) | (1u << WL_K_PROLONG) | (1u << WL_K_COARSE) | (1u << WL_K_REDUCE);
    return !prof.on || (prof.groups & inside) == 0;
  }

  // vcycle(0), through a cached graph where one matches (else captured, then
  // launched); plain launches where graphs are not allowed.  A failed capture
  // turns graphs off for the sim (for instance when the caller is itself
  // capturing the sim's stream).
  wl_status vcycle_top() {
    if (!vcg_allowed()) {
      vcycle(0);
      return WL_OK;
    }
    const size_t bbytes = sizeof(StdBox) * (size_t)nlev;
    for (auto& gr : vcg)
      if (gr.valid && std::memcmp(gr.pre, slot_n, sizeof(slot_n)) == 0 && std::memcmp(gr.box, sbox, bbytes) == 0) {
        WL_HIP(hipGraphLaunch(gr.exec, stream));
        std::memcpy(slot_n, gr.post, sizeof(slot_n));
        return WL_OK;
      }
    int pre[kNumSlots];
    std::memcpy(pre, slot_n, sizeof(slot_n));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t he = hipSuccess;
    if (!cap_stream) he = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
      hipStream_t own = stream;
      stream = cap_stream;  // every launch of the cycle goes to the capture
      vcycle(0);
      stream = own;
      he = hipStreamEndCapture(cap_stream, &graph);
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (he != hipSuccess) {
      // nothing of the captured cycle ran: plain launches from here on
      (void)hipGetLastError();
      vcg_off = true;
      std::memcpy(slot_n, pre, sizeof(slot_n));
      vcycle(0);
      return WL_OK;
    }
    VcGraph& gr = vcg[vcg_next];
    vcg_next = (vcg_next + 1) % kVcGraphs;
    if (gr.valid && gr.exec) (void)hipGraphExecDestroy(gr.exec);
    gr.valid = true;
    gr.exec = exec;
    std::memcpy(gr.pre, pre, sizeof(pre));
    std::memcpy(gr.post, slot_n, sizeof(slot_n));
    std::memcpy(gr.box, sbox, bbytes);
    WL_HIP(hipGraphLaunch(exec, stream));
    return WL_OK;
  }

  ~Impl() override {
    for (auto& gr : vcg)
      if (gr.valid && gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }

  void vcycle(int l) {
    if (nflat[l + 1] > 0) {
      const int nf = (int)nflat[l + 1];
      const bool direct = nf <= kFlatDirectMax && desc.reduce_mode == 0;
      double* const psum = direct ? slot(kSlotSumR) : wide;
      double* const pcnt = direct ? slot(kSlotCnt) : wide + wide_n;
      if (desc.periodic_mask)
        {
          if (l == 0)
            WL_TIMED(l == 0 ? WL_K_RESTRICT : WL_K_COARSE,
                     (k_restrict_flat<T, true, 1><<<flat_grid(l + 1), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], r[l], iD[l + 1], r[l + 1], x[l + 1], psum, pcnt, flags + l + 1, sbox[l + 1])));
          else
            WL_TIMED(l == 0 ? WL_K_RESTRICT : WL_K_COARSE,
                     (k_restrict_flat<T, true, 0><<<flat_grid(l + 1), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], r[l], iD[l + 1], r[l + 1], x[l + 1], psum, pcnt, flags + l + 1, sbox[l + 1])));
        }
      else
        {
          if (l == 0)
            WL_TIMED(l == 0 ? WL_K_RESTRICT : WL_K_COARSE,
                     (k_restrict_flat<T, false, 1><<<flat_grid(l + 1), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], r[l], iD[l + 1], r[l + 1], x[l + 1], psum, pcnt, flags + l + 1, sbox[l + 1])));
          else
            WL_TIMED(l == 0 ? WL_K_RESTRICT : WL_K_COARSE,
                     (k_restrict_flat<T, false, 0><<<flat_grid(l + 1), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], r[l], iD[l + 1], r[l + 1], x[l + 1], psum, pcnt, flags + l + 1, sbox[l + 1])));
        }
      if (direct)
        set_mean_producer(nf);
      else
        reduce_wide(psum, 0, pcnt, 0, nf, kSlotSumR, kSlotCnt);
    } else {
      WL_TIMED(l == 0 ? WL_K_RESTRICT : WL_K_COARSE,
               (k_restrict<T, D><<<nb[l + 1], kBlock, 0, stream>>>(g[l], g[l + 1], r[l], iD[l + 1], r[l + 1],
                                                                   x[l + 1], red, flags + l + 1)));
      set_mean_producer(nb[l + 1]);
    }
    if (l + 1 == lbot) {
      bottom(l + 1);  // the rest of the cycle below, and PCG on level l+1
    } else {
      if (l + 2 < nlev) vcycle(l + 1);
      pcg(l + 1, false);
    }
    if (nflat[l] > 0) {
      const int nf = (int)nflat[l];
      const bool direct = nf <= kFlatDirectMax && desc.reduce_mode == 0;
      double* const psum = direct ? slot(kSlotSumR) : wide;
      double* const pcnt = direct ? slot(kSlotCnt) : wide + wide_n;
      if (desc.periodic_mask)
        {
          if (l == 0)
            WL_TIMED(l == 0 ? WL_K_PROLONG : WL_K_COARSE,
                     (k_prolong_flat<T, true, 1><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], x[l + 1], v3(L[l]), iD[l], x[l], r[l], psum, pcnt, flags + l, sbox[l])));
          else
            WL_TIMED(l == 0 ? WL_K_PROLONG : WL_K_COARSE,
                     (k_prolong_flat<T, true, 0><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], x[l + 1], v3(L[l]), iD[l], x[l], r[l], psum, pcnt, flags + l, sbox[l])));
        }
      else
        {
          if (l == 0)
            WL_TIMED(l == 0 ? WL_K_PROLONG : WL_K_COARSE,
                     (k_prolong_flat<T, false, 1><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], x[l + 1], v3(L[l]), iD[l], x[l], r[l], psum, pcnt, flags + l, sbox[l])));
          else
            WL_TIMED(l == 0 ? WL_K_PROLONG : WL_K_COARSE,
                     (k_prolong_flat<T, false, 0><<<flat_grid(l), kFlatThreads, 0, stream>>>(
                         g[l], g[l + 1], x[l + 1], v3(L[l]), iD[l], x[l], r[l], psum, pcnt, flags + l, sbox[l])));
        }
      if (direct)
        set_mean_producer(nf);
      else
        reduce_wide(psum, 0, pcnt, 0, nf, kSlotSumR, kSlotCnt);
    } else if (tiles[l][2] > 0) {
      WL_TIMED(l == 0 ? WL_K_PROLONG : WL_K_COARSE,
               (k_prolong_tile<T><<<tiles[l][2], kTileThreads, 0, stream>>>(
                   g[l], g[l + 1], x[l + 1], v3(L[l]), iD[l], x[l], r[l], red, flags + l, tiles[l][0],
                   tiles[l][1], tiles[l][2], tiles[l][3], sbox[l])));
      set_mean_producer(tiles[l][2]);
    } else {
      WL_TIMED(l == 0 ? WL_K_PROLONG : WL_K_COARSE,
               (k_prolong<T, D><<<nb[l], kBlock, 0, stream>>>(g[l], g[l + 1], x[l + 1], v3(L[l]), iD[l], x[l],
                                                              r[l], red, flags + l)));
      set_mean_producer(nb[l]);
    }
  }

  // squared 2-norm of the fine residual (FP64 sum over the interior) into scal[kScalL2 + which]
  void res_sumsq(int which) {
    const int nf = (int)nflat[0];
    if (D == 3 && nf > 0) {
      WL_TIMED(WL_K_REDUCE, (k_sumsq_flat<T><<<flat_grid(0), kFlatThreads, 0, stream>>>(g[0], r[0], wide)));
      reduce_wide(wide, 0, nullptr, 0, nf, kSlotL2, -1);
      WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(slot(kSlotL2), 0, nullptr, 0, 1,
                                                                             scal + kScalL2 + which, nullptr)));
      return;
    }
    const int rows = g[0].n[1] * (D == 3 ? g[0].n[2] : 1);
    const int gb = std::min(rows, kGridStride);
    WL_TIMED(WL_K_REDUCE, (k_sumsq<T, D><<<gb, kBlock, 0, stream>>>(g[0], r[0], slot(kSlotL2))));
    WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(slot(kSlotL2), 0, nullptr, 0, gb,
                                                                           scal + kScalL2 + which, nullptr)));
  }

  // initial residual already in r[0] / rmax slot.  l2_which 0/1: the residual's
  // 2-norm is left in scal for the step to read with its other scalars; -1: read now.
  wl_status mg_loop(double tol, int itmax, wl_solve_stats* st, int l2_which = -1) {
    double res0;
    wl_status s = read_scalar_max(kSlotRmax, &res0);
    if (s != WL_OK) return s;
    double res = res0;
    int n = 0;
    while (res >= tol && n < itmax) {
      if (nlev > 1) {
        if ((s = vcycle_top()) != WL_OK) return s;
      }
      else {
        WL_TIMED(WL_K_DIVRES, (k_mean0<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], iD[0], r[0], red, flags)));
        set_mean_producer(nb[0]);
      }
      pcg(0, true);
      ++n;
      s = read_scalar_max(kSlotRmax, &res);
      if (s != WL_OK) return s;
      if (!std::isfinite(res)) return fail(WL_ERR_NONFINITE, "multigrid residual is not finite");
    }
    if (!std::isfinite(res0)) return fail(WL_ERR_NONFINITE, "initial residual is not finite");
    res_sumsq(l2_which < 0 ? 0 : l2_which);
    WL_HIP(hipGetLastError());
    double l2 = NAN;
    if (l2_which < 0) {
      WL_HIP(hipMemcpyAsync(host_pin, scal + kScalL2, sizeof(double), hipMemcpyDeviceToHost, stream));
      WL_HIP(hipStreamSynchronize(stream));
      prof.harvest();
      l2 = std::sqrt(host_pin[0]);
    }
    if (st) {
      st->vcycles = n;
      st->res0_linf = res0;
      st->res_linf = res;
      st->res_l2 = l2;
      st->converged = res < tol ? 1 : 0;
    }
    return WL_OK;
  }

  // divergence (or rhs), warm start and initial residual on the fine level; leaves
  // the max|r| and mean partials with their counts set
  void div_res(T* const uu[3], const T* rhs, const T* pp, T wdt) {
    const int nf = (int)nflat[0];
    // the flat kernel reads rhs in 16-byte vectors starting at x = 1: a caller's
    // array without the fields' front padding takes the generic kernel
    const bool aligned = rhs == nullptr || (reinterpret_cast<uintptr_t>(rhs + 1) % 16) == 0;
    if (nf > 0 && aligned) {
      const bool direct = nf <= kFlatDirectMax && desc.reduce_mode == 0;
      double* const pmax = direct ? slot(kSlotRmax) : wide;
      double* const psum = direct ? slot(kSlotSumR) : wide + wide_n;
      double* const pcnt = direct ? slot(kSlotCnt) : wide + 2 * wide_n;
      if (desc.periodic_mask)
        WL_TIMED(WL_K_DIVRES, (k_div_res_flat<T, true><<<flat_grid(0), kFlatThreads, 0, stream>>>(
                                  g[0], v3(uu), rhs, pp, wdt, v3(L[0]), iD[0], x[0], r[0], pmax, psum, pcnt, flags,
                                  sbox[0])));
      else
        WL_TIMED(WL_K_DIVRES, (k_div_res_flat<T, false><<<flat_grid(0), kFlatThreads, 0, stream>>>(
                                  g[0], v3(uu), rhs, pp, wdt, v3(L[0]), iD[0], x[0], r[0], pmax, psum, pcnt, flags,
                                  sbox[0])));
      if (direct) {
        slot_n[kSlotRmax] = nf;
        set_mean_producer(nf);
      } else {
        reduce_wide(psum, 0, pcnt, 0, nf, kSlotSumR, kSlotCnt);
        reduce_wide(pmax, 1, nullptr, 0, nf, kSlotRmax, -1);
      }
    } else {
      WL_TIMED(WL_K_DIVRES, (k_div_res<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], v3(uu), rhs, pp, wdt, v3(L[0]),
                                                                            iD[0], x[0], r[0], slot(kSlotRmax), red,
                                                                            flags, sbox[0])));
      slot_n[kSlotRmax] = nb[0];
      set_mean_producer(nb[0]);
    }
  }

  wl_status project(T* const uu[3], double w, wl_solve_stats* st, int l2_which = -1) {
    const T wdt = T(w * dt);
    const bool guided = pg_on && pg_mode >= 1 && pg_hist >= 2;
    if (guided) {
      // multigrid decides on the guess: it is used only if its initial residual is below
      // that of the plain warm start x0 = p w dt
      double res_plain = 0.0, res_guess = 0.0;
      div_res(uu, nullptr, p, wdt);
      wl_status s0 = read_scalar_max(kSlotRmax, &res_plain);
      if (s0 != WL_OK) return s0;
      pg_guess(uu, w * dt);  // x[0] = learned guess
      div_res(uu, nullptr, nullptr, wdt);
      if ((s0 = read_scalar_max(kSlotRmax, &res_guess)) != WL_OK) return s0;
      ++pg_tried;
      if (res_guess < res_plain) {
        ++pg_used;
      } else {
        div_res(uu, nullptr, p, wdt);
      }
    } else {
      div_res(uu, nullptr, p, wdt);
    }
    WL_HIP(hipGetLastError());
    wl_status s = mg_loop(desc.mg_tol, desc.mg_itmax, st, l2_which);
    if (s != WL_OK) return s;
    if (guided && pg_mode == 2) pg_snapshot(w * dt);
    if (pg_on) WL_HIP(hipMemcpyAsync(p2, p, plan.lev[0].elems * sizeof(T), hipMemcpyDeviceToDevice, stream));
    if (nflat[0] > 0) {
      if (desc.periodic_mask)
        WL_TIMED(WL_K_PROJECT, (k_project_flat<T, true><<<flat_grid(0), kFlatThreads, 0, stream>>>(
                                   g[0], v3(uu), v3(L[0]), x[0], p, wdt, sbox[0])));
      else
        WL_TIMED(WL_K_PROJECT, (k_project_flat<T, false><<<flat_grid(0), kFlatThreads, 0, stream>>>(
                                   g[0], v3(uu), v3(L[0]), x[0], p, wdt, sbox[0])));
    } else {
      WL_TIMED(WL_K_PROJECT, (k_project<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], v3(uu), v3(L[0]), x[0], p, wdt,
                                                                            sbox[0])));
    }
    WL_HIP(hipGetLastError());
    if (pg_on) ++pg_hist;
    if (pg_on && pg_mode == 2 && ring_used > 0) {
      for (int k = 0; k < pg_iters; ++k) {
        const int slot_k = (int)(next_rand() % (uint64_t)ring_used);
        pg_train_box(bcrop, ringX[slot_k], ringT[slot_k], ringM[slot_k], true);
      }
    }
    return WL_OK;
  }

  // ---- learned initial guess --------------------------------------------------
  uint64_t next_rand() {  // SplitMix64 stream
    uint64_t z = (pg_rng += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }

  void pg_net(const PgBox& b, const unsigned short* X, unsigned short* a1, unsigned short* a2, float* y, int kid) {
    const int64_t tasks = (int64_t)((b.n[0] + 15) / 16) * b.n[1] * b.n[2];
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tasks + 3) / 4, kGridStride));
    WL_TIMED(kid, (k_pg_conv<4, 0><<<grid, kBlock, 0, stream>>>(b, X, pgK.w1f, pgK.b1, a1, nullptr, nullptr)));
    WL_TIMED(kid, (k_pg_conv<16, 0><<<grid, kBlock, 0, stream>>>(b, a1, pgK.w2f, pgK.b2, a2, nullptr, nullptr)));
    WL_TIMED(kid, (k_pg_conv<16, 1><<<grid, kBlock, 0, stream>>>(b, a2, pgK.w3f, pgK.b3, nullptr, y, nullptr)));
  }

  void pg_guess(T* const uu[3], double wdt) {
    WL_TIMED(WL_K_PG_INFER, (k_pg_moments<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], p, iD[0], pgRed)));
    WL_TIMED(WL_K_PG_INFER, (k_pg_norm<<<1, kBlock, 0, stream>>>(pgRed, nb[0], pgScal)));
    WL_TIMED(WL_K_PG_INFER, (k_pg_features<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], bd, v3(uu), p, p2, iD[0],
                                                                                pgScal, wdt, pgXd)));
    pg_net(bd, pgXd, pgA1d, pgA2d, pgYd, WL_K_PG_INFER);
    WL_TIMED(WL_K_PG_INFER, (k_pg_guess<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], bd, p, iD[0], pgYd, pgScal, wdt,
                                                                             x[0])));
  }

  void pg_snapshot(double wdt) {
    for (int c = 0; c < pg_crops; ++c) {
      int o[3];
      for (int a = 0; a < 3; ++a) o[a] = 1 + (int)(next_rand() % (uint64_t)(bd.n[a] - bcrop.n[a] + 1));
      const int k = ring_next;
      WL_TIMED(WL_K_PG_TRAIN, (k_pg_crop<T, D><<<blocks_for((int64_t)bcrop.n[0] * bcrop.n[1] * bcrop.n[2]), kBlock, 0, stream>>>(
                                  g[0], bd, pgXd, x[0], p, iD[0], pgScal, wdt, o[0], o[1], o[2], bcrop, ringX[k], ringT[k],
                                  ringM[k])));
      ring_next = (ring_next + 1) % kPgRing;
      ring_used = std::min(ring_used + 1, kPgRing);
      ++pg_snaps;
    }
  }

  // forward + loss + backward on a box (the crop buffers hold the activations);
  // gradient into pgGrad, Adam step if apply
  void pg_train_box(const PgBox& b, const unsigned short* X, const float* tgt, const unsigned char* msk, bool apply) {
    const int K = WL_K_PG_TRAIN;
    pg_net(b, X, pgA1c, pgA2c, pgYc, K);
    const int gb = blocks_for((int64_t)b.n[0] * b.n[1] * b.n[2]);
    WL_TIMED(K, (k_pg_err<<<gb, kBlock, 0, stream>>>(b, pgYc, tgt, msk, pgRed)));
    WL_TIMED(K, (k_pg_dy<<<gb, kBlock, 0, stream>>>(b, pgYc, tgt, msk, pgRed, gb, pgG3, pgRed + 4096)));
    pg_loss_blocks = gb;
    pg_loss_pending = true;
    const int64_t tasks = (int64_t)((b.n[0] + 15) / 16) * b.n[1] * b.n[2];
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tasks + 3) / 4, kGridStride));
    WL_TIMED(K, (k_pg_conv<16, 2><<<grid, kBlock, 0, stream>>>(b, pgG3, pgK.w3b, nullptr, pgG2, nullptr, pgA2c)));
    WL_TIMED(K, (k_pg_conv<16, 2><<<grid, kBlock, 0, stream>>>(b, pgG2, pgK.w2b, nullptr, pgG1, nullptr, pgA1c)));
    const int wb = kPgWaves / 4;
    WL_TIMED(K, (k_pg_wgrad<16><<<wb, kBlock, 0, stream>>>(b, pgA2c, pgG3, pgPart)));
    WL_TIMED(K, (k_pg_wgrad_reduce<<<32, kBlock, 0, stream>>>(pgPart, kPgWaves, 16, 1, pgGrad + kPgW3, pgGrad + kPgB3)));
    WL_TIMED(K, (k_pg_wgrad<16><<<wb, kBlock, 0, stream>>>(b, pgA1c, pgG2, pgPart)));
    WL_TIMED(K, (k_pg_wgrad_reduce<<<32, kBlock, 0, stream>>>(pgPart, kPgWaves, 16, 16, pgGrad + kPgW2, pgGrad + kPgB2)));
    WL_TIMED(K, (k_pg_wgrad<4><<<wb, kBlock, 0, stream>>>(b, X, pgG1, pgPart)));
    WL_TIMED(K, (k_pg_wgrad_reduce<<<32, kBlock, 0, stream>>>(pgPart, kPgWaves, 3, 16, pgGrad + kPgW1, pgGrad + kPgB1)));
    ++pg_train_steps;
    if (apply) {
      ++pg_adam_t;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.f - (float)std::pow(0.9, (double)pg_adam_t), c2 = 1.f - (float)std::pow(0.999, (double)pg_adam_t);
      WL_TIMED(K, (k_pg_adam<<<blocks_for(kPgParams), kBlock, 0, stream>>>(pgW, pgM, pgV, pgGrad, (float)pg_lr, b1, b2,
                                                                           c1, c2, 1e-8f, 1)));
      WL_TIMED(K, (k_pg_pack<<<blocks_for(27 * 256), kBlock, 0, stream>>>(pgW, pgK)));
    }
  }
  int pg_loss_blocks = 0;

  wl_status pg_require() const {
    if (!pg_on) return fail(WL_ERR_UNSUPPORTED, "learned guess needs desc.learned_guess = 1 and ndim = 3");
    return WL_OK;
  }

  wl_status pg_set_weights(const float* w) override {
    if (pg_require() != WL_OK) return WL_ERR_UNSUPPORTED;
    if (!w) return fail(WL_ERR_INVALID_ARG, "weights are NULL");
    for (int k = 0; k < kPgParams; ++k)
      if (!std::isfinite(w[k])) return fail(WL_ERR_INVALID_ARG, "weights must be finite");
    WL_HIP(hipMemcpyAsync(pgW, w, kPgParams * sizeof(float), hipMemcpyHostToDevice, stream));
    WL_HIP(hipMemsetAsync(pgM, 0, kPgParams * sizeof(float), stream));
    WL_HIP(hipMemsetAsync(pgV, 0, kPgParams * sizeof(float), stream));
    k_pg_pack<<<blocks_for(27 * 256), kBlock, 0, stream>>>(pgW, pgK);
    WL_HIP(hipGetLastError());
    WL_HIP(hipStreamSynchronize(stream));
    pg_adam_t = 0;
    pg_weights_set = true;
    return WL_OK;
  }

  wl_status pg_get_weights(float* w) override {
    if (pg_require() != WL_OK) return WL_ERR_UNSUPPORTED;
    if (!w) return fail(WL_ERR_INVALID_ARG, "output is NULL");
    WL_HIP(hipMemcpyAsync(w, pgW, kPgParams * sizeof(float), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    return WL_OK;
  }

  wl_status pg_set_mode(int mode, double lr, int iters, int crops, uint64_t seed) override {
    if (pg_require() != WL_OK) return WL_ERR_UNSUPPORTED;
    if (mode < 0 || mode > 2 || !(lr >= 0.0) || iters < 0 || crops < 0 || crops > kPgRing)
      return fail(WL_ERR_INVALID_ARG, "mode in 0..2, lr >= 0, iters >= 0, crops in 0..64");
    if (mode >= 1 && !pg_weights_set) return fail(WL_ERR_INVALID_ARG, "set the weights before enabling the guess");
    pg_mode = mode;
    pg_lr = lr;
    pg_iters = iters;
    pg_crops = crops;
    pg_rng = seed;
    return WL_OK;
  }

  wl_status pg_box(const int64_t n[3], PgBox& b) const {
    if (!n) return fail(WL_ERR_INVALID_ARG, "box size is NULL");
    for (int a = 0; a < 3; ++a) {
      if (n[a] < 1 || n[a] > bcrop.n[a]) return fail(WL_ERR_INVALID_ARG, "box must fit the training crop");
      b.n[a] = (int)n[a];
      b.P[a] = b.n[a] + 2;
    }
    return WL_OK;
  }

  wl_status pg_forward(const void* xin, const int64_t n[3], float* y) override {
    if (pg_require() != WL_OK) return WL_ERR_UNSUPPORTED;
    PgBox b;
    if (pg_box(n, b) != WL_OK) return WL_ERR_INVALID_ARG;
    if (!xin || !y) return fail(WL_ERR_INVALID_ARG, "box arrays are NULL");
    WL_HIP(hipMemsetAsync(pgA1c, 0, (size_t)pgPc * 32, stream));
    WL_HIP(hipMemsetAsync(pgA2c, 0, (size_t)pgPc * 32, stream));
    pg_net(b, (const unsigned short*)xin, pgA1c, pgA2c, y, WL_K_PG_INFER);
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  wl_status read_loss() {
    if (!pg_loss_pending) return WL_OK;
    std::vector<double> h(pg_loss_blocks);
    WL_HIP(hipMemcpyAsync(h.data(), pgRed + 4096, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    double l = 0;
    for (double v : h) l += v;
    pg_last_loss = l;
    pg_loss_pending = false;
    return WL_OK;
  }

  wl_status pg_train(const void* xin, const float* tg, const unsigned char* mk, const int64_t n[3], float* grad,
                     double* loss, int apply) override {
    if (pg_require() != WL_OK) return WL_ERR_UNSUPPORTED;
    PgBox b;
    if (pg_box(n, b) != WL_OK) return WL_ERR_INVALID_ARG;
    if (!xin || !tg || !mk) return fail(WL_ERR_INVALID_ARG, "box arrays are NULL");
    if (!pg_weights_set) return fail(WL_ERR_INVALID_ARG, "set the weights first");
    // box layout differs from the crop layout: clear the halos of the activation buffers
    for (unsigned short* bptr : {pgA1c, pgA2c, pgG3, pgG2, pgG1})
      WL_HIP(hipMemsetAsync(bptr, 0, (size_t)pgPc * 32, stream));
    pg_train_box(b, (const unsigned short*)xin, tg, mk, apply != 0);
    WL_HIP(hipGetLastError());
    if (grad) {
      WL_HIP(hipMemcpyAsync(grad, pgGrad, kPgParams * sizeof(float), hipMemcpyDeviceToHost, stream));
    }
    wl_status s = read_loss();
    if (s != WL_OK) return s;
    if (loss) *loss = pg_last_loss;
    // restore clean crop-layout buffers for the online training
    for (unsigned short* bptr : {pgA1c, pgA2c, pgG3, pgG2, pgG1})
      WL_HIP(hipMemsetAsync(bptr, 0, (size_t)pgPc * 32, stream));
    WL_HIP(hipStreamSynchronize(stream));
    return WL_OK;
  }

  wl_status pg_stats(double* loss, int64_t* steps, int64_t* snaps, int64_t* used, int64_t* tried) override {
    if (pg_require() != WL_OK) return WL_ERR_UNSUPPORTED;
    wl_status s = read_loss();
    if (s != WL_OK) return s;
    if (loss) *loss = pg_last_loss;
    if (steps) *steps = pg_train_steps;
    if (snaps) *snaps = pg_snaps;
    if (used) *used = pg_used;
    if (tried) *tried = pg_tried;
    return WL_OK;
  }

  wl_status project_cur(double w, wl_solve_stats* st) override {
    wl_status s = project(u[cur], w, st);
    if (s != WL_OK) return s;
    return bc(u[cur], false);
  }

  wl_status poisson(const void* rhs, void* xin, double tol, int itmax, wl_solve_stats* st) override {
    // a caller-supplied x (pressure layout, no front padding) is copied in and out of
    // the internal fine-level x, which the vectorised kernels require
    const size_t bytes = (size_t)plan.lev[0].elems * sizeof(T);
    if (xin) WL_HIP(hipMemcpyAsync(x[0], xin, bytes, hipMemcpyDeviceToDevice, stream));
    div_res(u[cur], (const T*)rhs, nullptr, T(0));
    WL_HIP(hipGetLastError());
    wl_status s = mg_loop(tol > 0 ? tol : desc.mg_tol, itmax > 0 ? itmax : desc.mg_itmax, st);
    if (s != WL_OK) return s;
    if (xin) WL_HIP(hipMemcpyAsync(xin, x[0], bytes, hipMemcpyDeviceToDevice, stream));
    return WL_OK;
  }

  // f~ = u0 + dt R(u) - V on every padded face (fuse = 0), or, in 3-D, the blend
  // of the predictor (fuse = 1) or the corrector (fuse = 2) written to uo outside
  // the body box and f~ kept near it (k_flux_reuse)
  wl_status flux(T* const uu[3], T* const uu0[3], int hb, int fuse = 0, T* const uo[3] = nullptr) {
    if (D == 3) {
      // output bricks of 63 columns x kRW rows x kRZ planes
      const int nbx = (g[0].n[0] + 2 + kRX - 2) / (kRX - 1), nby = (g[0].n[1] + 2 + kRW - 1) / kRW,
                nbz = (g[0].n[2] + 2 + kRZ - 1) / kRZ;
      const dim3 grid(nbx * nby * nbz * 3);
      const Vec3<T> o = v3(uo ? uo : ft);
      if (fuse == 1)
        WL_TIMED(WL_K_FLUX, (k_flux_reuse<T, 1><<<grid, kReuseThreads, 0, stream>>>(
                                g[0], v3(uu), v3(uu0), v3(V), v3(ft), o, T(dt), T(desc.nu), hb, sbox[0], nbx, nby, nbz)));
      else if (fuse == 2)
        WL_TIMED(WL_K_FLUX, (k_flux_reuse<T, 2><<<grid, kReuseThreads, 0, stream>>>(
                                g[0], v3(uu), v3(uu0), v3(V), v3(ft), o, T(dt), T(desc.nu), hb, sbox[0], nbx, nby, nbz)));
      else
        WL_TIMED(WL_K_FLUX, (k_flux_reuse<T, 0><<<grid, kReuseThreads, 0, stream>>>(
                                g[0], v3(uu), v3(uu0), v3(V), v3(ft), o, T(dt), T(desc.nu), hb, sbox[0], nbx, nby, nbz)));
    } else {
      WL_TIMED(WL_K_FLUX, (k_flux<T, D><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                              g[0], v3(uu), v3(uu0), v3(V), v3(ft), T(dt), T(desc.nu), hb, 0, sbox[0])));
    }
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  // max over the cells of the CFL sum and of |div u| over the active cells, into
  // scal (kScalCfl, kScalDiv): flat vectors on a 3-D fine level that takes them
  wl_status cfl_max() {
    const int nf = (int)nflat[0];
    if (D == 3 && nf > 0) {
      double* const pa = wide;
      double* const pb = wide + wide_n;
      if (desc.periodic_mask)
        WL_TIMED(WL_K_CFL, (k_cfl_flat<T, true><<<flat_grid(0), kFlatThreads, 0, stream>>>(
                               g[0], v3(u[cur]), iD[0], sbox[0], pa, pb)));
      else
        WL_TIMED(WL_K_CFL, (k_cfl_flat<T, false><<<flat_grid(0), kFlatThreads, 0, stream>>>(
                               g[0], v3(u[cur]), iD[0], sbox[0], pa, pb)));
      reduce_wide(pa, 1, pb, 1, nf, kSlotCfl, kSlotDiv);
      WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(slot(kSlotCfl), 1, slot(kSlotDiv), 1, 1,
                                                                             scal + kScalCfl, scal + kScalDiv)));
    } else {
      WL_TIMED(WL_K_CFL, (k_cfl<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], v3(u[cur]), iD[0], sbox[0],
                                                                      slot(kSlotCfl), slot(kSlotDiv))));
      WL_TIMED(WL_K_REDUCE, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(
                                slot(kSlotCfl), 1, slot(kSlotDiv), 1, nb[0], scal + kScalCfl, scal + kScalDiv)));
    }
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  // blend of the body box's faces after a fused flux launch: uo from f~ and, for
  // the corrector, this stage's velocity uu (nothing to do without a body box)
  wl_status bdim_box(int corr, T* const uu[3], T* const uo[3]) {
    const StdBox& Bx = sbox[0];
    if (!has_body || Bx.lo[0] > Bx.hi[0]) return WL_OK;
    int lo[3], cnt[3];
    int64_t vol = 1;
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::max(Bx.lo[a], 0);
      cnt[a] = std::min(Bx.hi[a], g[0].n[a] + 1) - lo[a] + 1;
      if (cnt[a] <= 0) return WL_OK;
      vol *= cnt[a];
    }
    const dim3 grid(blocks_for(vol), D);
    const int3 l3 = make_int3(lo[0], lo[1], lo[2]), n3 = make_int3(cnt[0], cnt[1], cnt[2]);
    if (corr)
      WL_TIMED(WL_K_BDIM, (k_bdim_box<T, 1><<<grid, kBlock, 0, stream>>>(g[0], v3(ft), v3(V), v3(mu0), v9(mu1), v3(uu),
                                                                        v3(uo), Bx, l3, n3)));
    else
      WL_TIMED(WL_K_BDIM, (k_bdim_box<T, 0><<<grid, kBlock, 0, stream>>>(g[0], v3(ft), v3(V), v3(mu0), v9(mu1), v3(uu),
                                                                        v3(uo), Bx, l3, n3)));
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  wl_status conv_diff() override {
    k_flux<T, D><<<dim3(nb_face, D), kBlock, 0, stream>>>(g[0], v3(u[cur]), v3(u[cur]), v3(V), v3(ft), T(0),
                                                          T(desc.nu), 0, 1, sbox[0]);
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  wl_status step(int remeasure, wl_step_stats* st) override {
    wl_status s;
    if (remeasure && moving) {
      s = remeasure_moving(t);
      if (s != WL_OK) return s;
    }
    T* const* A = u[cur];
    T* const* B = u[1 - cur];
    const int hb = has_body ? 1 : 0;
    // 3-D steps that record nothing for the adjoint blend in the flux launch away
    // from the body; the corrector then writes u^{n+1} over u^n (A), which only the
    // flux launch itself reads, face by face, and the buffers do not swap
    const bool fuse = D == 3 && !rec && desc.blend_mode == 0;
    T* const* C = fuse ? A : B;  // the corrector's output
    // predictor
    if (fuse) {
      if ((s = flux(A, A, hb, 1, B)) != WL_OK) return s;
      if ((s = bdim_box(0, B, B)) != WL_OK) return s;
    } else {
      if ((s = flux(A, A, hb)) != WL_OK) return s;
      if (nflat[0] > 0)
        WL_TIMED(WL_K_BDIM, (k_bdim_flat<T, 0><<<bdim_grid(), kFlatThreads, 0, stream>>>(
                                g[0], v3(ft), v3(V), v3(mu0), v9(mu1), v3(B), hb, sbox[0])));
      else
        WL_TIMED(WL_K_BDIM, (k_bdim<T, D, 0><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                                g[0], v3(ft), v3(V), v3(mu0), v9(mu1), v3(B), hb, sbox[0])));
    }
    const bool ex = desc.convective_exit != 0;
    if (ex) {
      const int m = g[0].n[1] * (D == 3 ? g[0].n[2] : 1);
      const int be = blocks_for(m);
      WL_TIMED(WL_K_EXIT, (k_exit_raw<T, D><<<be, kBlock, 0, stream>>>(g[0], A[0], ebuf, T(dt * desc.U[0]),
                                                                      slot(kSlotExit))));
      const double inlet = double(m) * double(T(desc.U[0]));
      WL_TIMED(WL_K_EXIT, (k_exit_shift<<<1, kBlock, 0, stream>>>(slot(kSlotExit), be, inlet, double(m), scal)));
      exit_valid = true;
    }
    WL_HIP(hipGetLastError());
    if ((s = bc(B, ex)) != WL_OK) return s;
    wl_solve_stats s1{}, s2{};
    if ((s = project(B, 1.0, &s1, 0)) != WL_OK) return s;
    if ((s = bc(B, ex)) != WL_OK) return s;
    if (rec) {  // intermediates the adjoint of this step reads
      for (int k = 0; k < D; ++k) {
        WL_HIP(copy_field(recB[k], B[k]));
        WL_HIP(copy_field(recF[k], ft[k]));
      }
      WL_HIP(copy_field(recX1, x[0]));
    }
    // corrector
    if (fuse) {
      if ((s = flux(B, A, hb, 2, C)) != WL_OK) return s;
      if ((s = bdim_box(1, B, C)) != WL_OK) return s;
    } else {
      if ((s = flux(B, A, hb)) != WL_OK) return s;
      if (nflat[0] > 0)
        WL_TIMED(WL_K_BDIM, (k_bdim_flat<T, 1><<<bdim_grid(), kFlatThreads, 0, stream>>>(
                                g[0], v3(ft), v3(V), v3(mu0), v9(mu1), v3(B), hb, sbox[0])));
      else
        WL_TIMED(WL_K_BDIM, (k_bdim<T, D, 1><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                                g[0], v3(ft), v3(V), v3(mu0), v9(mu1), v3(B), hb, sbox[0])));
    }
    WL_HIP(hipGetLastError());
    if ((s = bc(C, ex)) != WL_OK) return s;
    if ((s = project(C, 0.5, &s2, 1)) != WL_OK) return s;
    if (rec) WL_HIP(copy_field(recX2, x[0]));
    if ((s = bc(C, ex)) != WL_OK) return s;
    if (!fuse) cur = 1 - cur;
    const double dt_used = dt;
    t += dt;
    // CFL (and the divergence check)
    if ((s = cfl_max()) != WL_OK) return s;
    WL_HIP(hipGetLastError());
    // one read-back for the step's scalars: the outflux maximum, both residual 2-norms
    // and the divergence check
    WL_HIP(hipMemcpyAsync(host_pin, scal, kNumScal * sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    prof.harvest();
    const double smax = host_pin[kScalCfl];
    s1.res_l2 = std::sqrt(host_pin[kScalL2]);
    s2.res_l2 = std::sqrt(host_pin[kScalL2 + 1]);
    const double div_linf = host_pin[kScalDiv];
    const double denom = smax + desc.cfl_nu_coef * desc.nu;
    dt = denom <= 0.0 ? desc.dt_max : std::min(desc.dt_max, 1.0 / denom);
    if (st) {
      st->dt = dt_used;
      st->t = t;
      st->dt_next = dt;
      st->vcycles[0] = s1.vcycles;
      st->vcycles[1] = s2.vcycles;
      st->res0_linf[0] = s1.res0_linf;
      st->res0_linf[1] = s2.res0_linf;
      st->res_linf[0] = s1.res_linf;
      st->res_linf[1] = s2.res_linf;
      st->res_l2[0] = s1.res_l2;
      st->res_l2[1] = s2.res_l2;
      st->div_linf = div_linf;
      st->converged = s1.converged && s2.converged;
    }
    if (!std::isfinite(smax) || !std::isfinite(dt)) return fail(WL_ERR_NONFINITE, "velocity is not finite");
    return WL_OK;
  }

  // the 11 force sums of the current state (k_forces partials, totalled in block order)
  wl_status force_sums(double tot[11]) {
    Motion m{};
    host_motion(parts, t, m);
    WL_TIMED(WL_K_FORCES, (k_forces<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], body, m, desc.eps, desc.nu,
                                                                         v3(u[cur]), p, iD[0],
                                                                         slot(kSlotForce), kMaxBlocks)));
    WL_HIP(hipGetLastError());
    std::vector<double> h((size_t)11 * kMaxBlocks);
    WL_HIP(hipMemcpyAsync(h.data(), slot(kSlotForce), h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    prof.harvest();
    for (int k = 0; k < 11; ++k) {
      double s_ = 0;
      for (int b = 0; b < nb[0]; ++b) s_ += h[(size_t)k * kMaxBlocks + b];
      tot[k] = s_;
    }
    return WL_OK;
  }

  wl_status forces(double fp[3], double fv[3]) override {
    for (int a = 0; a < 3; ++a) fp[a] = fv[a] = 0.0;
    if (!has_body) return WL_OK;
    double tot[11];
    wl_status s = force_sums(tot);
    if (s != WL_OK) return s;
    const double cnt = tot[10];
    const double pbar = cnt > 0 ? tot[9] / cnt : 0.0;
    for (int a = 0; a < 3; ++a) {
      fp[a] = -(tot[a] - pbar * tot[6 + a]);
      fv[a] = tot[3 + a];
    }
    return WL_OK;
  }

  // wl_forces with its partial sums in the caller-free scratch array (scr: that
  // array's device address): partials, their totals on the device, one 11-double
  // read-back into the pinned buffer.  No allocation of any kind.
  wl_status forces_static(double* scr, double fp[3], double fv[3]) override {
    for (int a = 0; a < 3; ++a) fp[a] = fv[a] = 0.0;
    if (!has_body) return WL_OK;
    if (nb[0] > kGridStride) return fail(WL_ERR_UNSUPPORTED, "force grid exceeds the static scratch");
    Motion m{};
    host_motion(parts, t, m);
    double* tot = scr + (size_t)kScratchRows * kGridStride;
    WL_TIMED(WL_K_FORCES, (k_forces<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], body, m, desc.eps, desc.nu,
                                                                         v3(u[cur]), p, iD[0], scr, kGridStride)));
    WL_TIMED(WL_K_FORCES, (k_sum_rows<<<kScratchRows, kBlock, 0, stream>>>(scr, nb[0], kGridStride, tot)));
    WL_HIP(hipGetLastError());
    WL_HIP(hipMemcpyAsync(host_pin, tot, kScratchRows * sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    prof.harvest();
    const double* h = host_pin;
    const double pbar = h[10] > 0 ? h[9] / h[10] : 0.0;
    for (int a = 0; a < 3; ++a) {
      fp[a] = -(h[a] - pbar * h[6 + a]);
      fv[a] = h[3 + a];
    }
    return WL_OK;
  }

  wl_status body_box_of(int level, int lo[3], int hi[3]) override {
    if (level < 0 || level >= nlev) return fail(WL_ERR_INVALID_ARG, "level out of range");
    for (int a = 0; a < 3; ++a) {
      lo[a] = sbox[level].lo[a];
      hi[a] = sbox[level].hi[a];
    }
    return WL_OK;
  }

  // ---- body update and discrete adjoint -----------------------------------------
  wl_status body_update(const wl_body_desc* b) override {
    if (!b) return fail(WL_ERR_INVALID_ARG, "body is NULL");
    std::vector<wl_body_desc> np;
    wl_status s = collect_parts(b, np);
    if (s != WL_OK) return s;
    // the workspace was planned for these parts: same count, kinds and sample grids
    bool same = np.size() == parts.size();
    for (size_t k = 0; same && k < np.size(); ++k) {
      same = np[k].kind == parts[k].kind && (np[k].vel_grid != nullptr) == plan.grid_vel[k];
      if (same && np[k].kind == WL_BODY_GRID_SDF)
        for (int a = 0; a < D; ++a) same = same && np[k].grid_n[a] == parts[k].grid_n[a];
    }
    if (!same) return fail(WL_ERR_INVALID_ARG, "the body's parts, kinds and sample grids cannot change");
    if ((s = validate_body(desc, b)) != WL_OK) return s;
    if (np.empty()) return WL_OK;
    parts = np;
    build_body();
    if ((s = upload_grids()) != WL_OK) return s;
    have_box = false;
    return measure(t);
  }

  // the adjoint needs a body whose shape does not move: every part static, except
  // spheres/circles that only spin about their centre
  wl_status adj_require() {
    if (!adj_on) return fail(WL_ERR_UNSUPPORTED, "the simulation has no adjoint buffers (desc.adjoint = 0)");
    if (desc.convective_exit) return fail(WL_ERR_UNSUPPORTED, "the adjoint does not cover the convective exit");
    for (const auto& p : parts) {
      wl_body_desc q = p;
      if (q.kind == WL_BODY_SPHERE && q.pivot_offset[0] == 0.0 && q.pivot_offset[1] == 0.0 && q.pivot_offset[2] == 0.0)
        q.spin_omega = 0.0;
      if (part_moving(q))
        return fail(WL_ERR_UNSUPPORTED,
                    "the adjoint needs a body whose shape does not move (spheres spinning about their centre are allowed)");
    }
    return WL_OK;
  }

  wl_status adj_reset() override {
    wl_status s = adj_require();
    if (s != WL_OK) return s;
    for (int k = 0; k < D; ++k) {
      fill_field(au[acur][k], T(0));
      fill_field(aVb[k], T(0));
      fill_field(am0b[k], T(0));
    }
    for (int k = 0; k < D * D; ++k) fill_field(am1b[k], T(0));
    fill_field(apb, T(0));
    WL_HIP(hipGetLastError());
    adj_dR = 0.0;
    return WL_OK;
  }

  void adj_bct(T* const w[3]) {
    for (int k = D - 1; k >= 0; --k) {
      int area = 1;
      for (int o = 0; o < D; ++o)
        if (o != k) area *= g[0].n[o] + 2;
      WL_TIMED(WL_K_ADJOINT,
               (k_adj_bc_axis<T, D><<<dim3(blocks_for(area), D), kBlock, 0, stream>>>(g[0], v3(w), k)));
    }
  }

  // transpose of project(w) + its velocity update: w = ubar of the projected
  // velocity in, of the unprojected velocity out; pbar (if with_p) consumed
  wl_status adj_project(T* const w[3], double wdt, const T* xs, bool with_p, double tol, wl_solve_stats* st) {
    WL_TIMED(WL_K_ADJOINT, (k_adj_proj_rhs<T, D><<<nb[0], kBlock, 0, stream>>>(
                               g[0], v3(w), v3(L[0]), with_p ? apb : nullptr, T(1.0 / wdt), iD[0], arhs)));
    fill_field(x[0], T(0));
    div_res(u[cur], arhs, nullptr, T(0));
    WL_HIP(hipGetLastError());
    wl_status s = mg_loop(tol, desc.mg_itmax, st);
    if (s != WL_OK) return s;
    WL_TIMED(WL_K_ADJOINT, (k_mean0<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], iD[0], x[0], red, flags)));
    set_mean_producer(nb[0]);
    int64_t faces = 1;
    for (int a = 0; a < D; ++a) faces *= g[0].n[a] + 1;
    WL_TIMED(WL_K_ADJOINT, (k_adj_proj_update<T, D><<<dim3(blocks_for(faces), D), kBlock, 0, stream>>>(
                               g[0], v3(w), x[0], xs, iD[0], v3(am0b), red, nb[0])));
    if (with_p) fill_field(apb, T(0));
    WL_HIP(hipGetLastError());
    return WL_OK;
  }

  wl_status adj_step(double tol, wl_step_stats* fst, wl_solve_stats* ast) override {
    return adj_step_impl(tol, false, 0, nullptr, fst, ast);
  }

  wl_status adj_step_cfl(double tol, int from_cfl, double* dtbar, wl_step_stats* fst,
                         wl_solve_stats* ast) override {
    return adj_step_impl(tol, true, from_cfl, dtbar, fst, ast);
  }

  // sum of per-block partials into red[kSlotForce*kMaxBlocks + k] (a slot the
  // multigrid solves never touch), k = 0..2
  void adj_total(const double* part, int n, int k) {
    WL_TIMED(WL_K_ADJOINT, (k_finalize2<<<1, kFinalizeThreads, 0, stream>>>(part, 0, nullptr, 0, n,
                                                                            slot(kSlotForce) + k, nullptr)));
  }

  // Reverse of one step (see wl_adj_step).  want_dt: also the adjoint of the step's
  // dt (returned in dtbar); from_cfl: dt came from the CFL rule of u^n, whose
  // transpose then adds dtbar d dt/du^n to the adjoint of u^n.
  wl_status adj_step_impl(double tol, bool want_dt, int from_cfl, double* dtbar, wl_step_stats* fst,
                          wl_solve_stats* ast) {
    wl_status s = adj_require();
    if (s != WL_OK) return s;
    const double dts = dt;  // the (frozen) step of the recomputed forward
    rec = true;
    s = step(1, fst);
    rec = false;
    if (s != WL_OK) return s;
    const double atol = tol > 0.0 ? tol : desc.mg_tol;
    T* const* A = u[1 - cur];     // u^n
    T* const* ub = au[acur];      // adjoint of u^{n+1}
    T* const* ua = au[1 - acur];  // becomes the adjoint of u^n
    const int hb = has_body ? 1 : 0;
    for (int k = 0; k < D; ++k) fill_field(ua[k], T(0));
    if (want_dt) {  // <pbar, p> of the state n+1, before the corrector's transpose consumes pbar
      WL_TIMED(WL_K_ADJOINT, (k_adj_dt_press<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], apb, p, slot(kSlotCfl))));
      adj_total(slot(kSlotCfl), nb[0], 0);
    }
    // corrector: bc, projection (w = 1/2, pbar), bc, blend (average), flux at the predictor state
    adj_bct(ub);
    if ((s = adj_project(ub, 0.5 * dts, recX2, true, atol, ast ? &ast[1] : nullptr)) != WL_OK) return s;
    adj_bct(ub);
    WL_TIMED(WL_K_ADJOINT, (k_adj_bdim<T, D, 1><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                               g[0], v3(ub), v3(ft), v3(mu0), v9(mu1), v3(afb), v3(aVb), v3(am0b), v9(am1b),
                               v3(aup), hb)));
    if (want_dt) {  // <fbar_2, f~_2 - u0 + V>
      WL_TIMED(WL_K_ADJOINT, (k_adj_dt_flux<T, D><<<nb_face, kBlock, 0, stream>>>(g[0], v3(afb), v3(ft), v3(A),
                                                                                   v3(V), slot(kSlotCfl))));
      adj_total(slot(kSlotCfl), nb_face, 1);
    }
    WL_TIMED(WL_K_ADJOINT, (k_adj_flux<T, D><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                               g[0], v3(recB), v3(afb), v3(aup), v3(ua), v3(aVb), T(dts), T(desc.nu), hb)));
    // predictor: bc, projection (w = 1), bc, blend, flux at u^n
    adj_bct(aup);
    if ((s = adj_project(aup, dts, recX1, false, atol, ast ? &ast[0] : nullptr)) != WL_OK) return s;
    adj_bct(aup);
    WL_TIMED(WL_K_ADJOINT, (k_adj_bdim<T, D, 0><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                               g[0], v3(aup), v3(recF), v3(mu0), v9(mu1), v3(afb), v3(aVb), v3(am0b), v9(am1b),
                               v3(aup), hb)));
    if (want_dt) {  // <fbar_1, f~_1 - u0 + V>
      WL_TIMED(WL_K_ADJOINT, (k_adj_dt_flux<T, D><<<nb_face, kBlock, 0, stream>>>(g[0], v3(afb), v3(recF), v3(A),
                                                                                   v3(V), slot(kSlotCfl))));
      adj_total(slot(kSlotCfl), nb_face, 2);
    }
    WL_TIMED(WL_K_ADJOINT, (k_adj_flux<T, D><<<dim3(nb_face, D), kBlock, 0, stream>>>(
                               g[0], v3(A), v3(afb), v3(ua), v3(ua), v3(aVb), T(dts), T(desc.nu), hb)));
    WL_HIP(hipGetLastError());
    if (want_dt) {
      WL_HIP(hipMemcpyAsync(host_pin, slot(kSlotForce), 3 * sizeof(double), hipMemcpyDeviceToHost, stream));
      WL_HIP(hipStreamSynchronize(stream));
      prof.harvest();
      const double db = (host_pin[1] + host_pin[2]) / dts - host_pin[0] / dts;
      if (dtbar) *dtbar = db;
      // dt_n = 1 / (sigma(I*) + 5 nu) of u^n when below dt_max
      if (from_cfl && dts < desc.dt_max) {
        WL_TIMED(WL_K_ADJOINT, (k_cfl_arg<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], v3(A), slot(kSlotCfl),
                                                                               slot(kSlotDiv))));
        WL_TIMED(WL_K_ADJOINT, (k_adj_cfl<T, D><<<1, kBlock, 0, stream>>>(g[0], v3(A), v3(ua), slot(kSlotCfl),
                                                                          slot(kSlotDiv), nb[0], -db * dts * dts)));
        WL_HIP(hipGetLastError());
      }
    }
    acur = 1 - acur;
    return WL_OK;
  }

  wl_status adj_forces(const double dir[3], double weight, double* value) override {
    wl_status s = adj_require();
    if (s != WL_OK) return s;
    if (!has_body) return fail(WL_ERR_INVALID_ARG, "no body: the force functional is 0");
    if (!dir || !std::isfinite(weight)) return fail(WL_ERR_INVALID_ARG, "dir is NULL or weight not finite");
    double tot[11];
    if ((s = force_sums(tot)) != WL_OK) return s;
    const double cnt = tot[10];
    const double pbar = cnt > 0 ? tot[9] / cnt : 0.0;
    double val = 0.0, nkm = 0.0;
    for (int a = 0; a < D; ++a) {
      val += dir[a] * (-(tot[a] - pbar * tot[6 + a]) + tot[3 + a]);
      nkm += dir[a] * (cnt > 0 ? tot[6 + a] / cnt : 0.0);
    }
    if (value) *value = val;
    Motion m{};
    host_motion(parts, t, m);
    const double3 d3 = make_double3(dir[0], dir[1], D == 3 ? dir[2] : 0.0);
    WL_TIMED(WL_K_ADJOINT, (k_adj_force_p<T, D><<<nb[0], kBlock, 0, stream>>>(g[0], body, m, desc.eps, iD[0], weight,
                                                                               d3, nkm, apb)));
    WL_TIMED(WL_K_ADJOINT, (k_adj_force_v<T, D><<<nb[0], kBlock, 0, stream>>>(
                               g[0], body, m, desc.eps, desc.nu, weight, d3, v3(u[cur]), p, pbar, v3(au[acur]),
                               slot(kSlotForce))));
    WL_HIP(hipGetLastError());
    std::vector<double> h((size_t)nb[0]);
    WL_HIP(hipMemcpyAsync(h.data(), slot(kSlotForce), h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    prof.harvest();
    for (double v : h) adj_dR += v;
    return WL_OK;
  }

  wl_status adj_body_grad(double* dR, double* dW) override {
    wl_status s = adj_require();
    if (s != WL_OK) return s;
    if (parts.size() != 1 || parts[0].kind != WL_BODY_SPHERE || body.general)
      return fail(WL_ERR_UNSUPPORTED, "body-parameter gradients need a single sphere/circle");
    Motion m{};
    host_motion(parts, t, m);
    const int gb = nb_face;
    WL_TIMED(WL_K_ADJOINT, (k_adj_body<T, D><<<dim3(gb, D), kBlock, 0, stream>>>(
                               g[0], body, m, desc.eps, v3(am0b), v9(am1b), v3(aVb), slot(kSlotForce))));
    WL_HIP(hipGetLastError());
    std::vector<double> h((size_t)6 * gb);
    WL_HIP(hipMemcpyAsync(h.data(), slot(kSlotForce), h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    WL_HIP(hipStreamSynchronize(stream));
    prof.harvest();
    double r_ = 0.0, w_ = 0.0;
    for (int c = 0; c < D; ++c)
      for (int b = 0; b < gb; ++b) {
        r_ += h[(size_t)c * gb + b];
        w_ += h[(size_t)(3 + c) * gb + b];
      }
    if (dR) *dR = r_ + adj_dR;
    if (dW) *dW = w_;
    return WL_OK;
  }

  wl_status field(int which, int level, void** ptr, int64_t shape[4], int64_t strides[4]) override {
    if (level < 0 || level >= nlev) return fail(WL_ERR_INVALID_ARG, "level out of range");
    const bool lev_field = which == WL_FIELD_X || which == WL_FIELD_R || which == WL_FIELD_L || which == WL_FIELD_ID;
    if (!lev_field && level != 0) return fail(WL_ERR_INVALID_ARG, "only X, R, L, ID have coarse levels");
    const LevelPlan& P = plan.lev[level];
    int ncomp = 1;
    T* base = nullptr;
    T* second = nullptr;
    switch (which) {
      case WL_FIELD_U: ncomp = D; base = u[cur][0]; second = D > 1 ? u[cur][1] : nullptr; break;
      case WL_FIELD_U0: ncomp = D; base = u[1 - cur][0]; second = u[1 - cur][1]; break;
      case WL_FIELD_F: ncomp = D; base = ft[0]; second = ft[1]; break;
      case WL_FIELD_V: ncomp = D; base = V[0]; second = V[1]; break;
      case WL_FIELD_MU0: ncomp = D; base = mu0[0]; second = mu0[1]; break;
      case WL_FIELD_MU1: ncomp = D * D; base = mu1[0]; second = mu1[1]; break;
      case WL_FIELD_P: base = p; break;
      case WL_FIELD_X: base = x[level]; break;
      case WL_FIELD_R: base = r[level]; break;
      case WL_FIELD_L: ncomp = D; base = L[level][0]; second = L[level][1]; break;
      case WL_FIELD_ID: base = iD[level]; break;
      case WL_FIELD_ADJ_U:
      case WL_FIELD_ADJ_P:
        if (!adj_on) return fail(WL_ERR_UNSUPPORTED, "the simulation has no adjoint buffers");
        if (which == WL_FIELD_ADJ_P) {
          base = apb;
        } else {
          ncomp = D;
          base = au[acur][0];
          second = au[acur][1];
        }
        break;
      default: return fail(WL_ERR_INVALID_ARG, "unknown field id");
    }
    *ptr = base;
    shape[0] = ncomp;
    shape[1] = P.pz;
    shape[2] = P.py;
    shape[3] = P.n[0] + 2;
    strides[0] = second ? (int64_t)(second - base) : 0;
    strides[1] = (int64_t)P.px * P.py;
    strides[2] = P.px;
    strides[3] = 1;
    return WL_OK;
  }
};

SimBase* make_impl(int prec, int ndim) {
  if (prec == WL_F32) return ndim == 2 ? (SimBase*)new Impl<float, 2>() : (SimBase*)new Impl<float, 3>();
  return ndim == 2 ? (SimBase*)new Impl<double, 2>() : (SimBase*)new Impl<double, 3>();
}

template <typename T, int D>
bool carve_impl(SimBase* s, void* ws, size_t bytes) {
  Impl<T, D>* im = static_cast<Impl<T, D>*>(s);
  const size_t used = im->carve((char*)ws);
  return used <= bytes && im->carved_ok((const char*)ws, bytes);
}

bool carve_any(SimBase* impl, const wl_sim_desc& d, void* ws, size_t bytes) {
  if (d.prec == WL_F32) return d.ndim == 2 ? carve_impl<float, 2>(impl, ws, bytes) : carve_impl<float, 3>(impl, ws, bytes);
  return d.ndim == 2 ? carve_impl<double, 2>(impl, ws, bytes) : carve_impl<double, 3>(impl, ws, bytes);
}

// Host-only dry run of the carving at a fake base address (never dereferenced).
bool plan_consistent(const wl_sim_desc& d, const Plan& P) {
  SimBase* impl = make_impl(d.prec, d.ndim);
  impl->desc = d;
  impl->plan = P;
  const bool ok = carve_any(impl, d, (void*)(uintptr_t)4096, P.bytes);
  delete impl;
  return ok;
}

// Device address of `scratch` on the current GPU, looked up once per device with
// that device current (the array's name is a host-side stand-in, never an address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

wl_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(WL_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(WL_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = (double*)g_scratch_dev[dev];
  return WL_OK;
}

}  // namespace

struct wl_sim {
  SimBase* impl;
};

extern "C" {

size_t wl_workspace_bytes(const wl_sim_desc* desc, const wl_body_desc* body) {
  wl_sim_desc d;
  if (validate_and_default(desc, &d) != WL_OK) return 0;
  if (validate_body(d, body) != WL_OK) return 0;
  std::vector<wl_body_desc> ps;
  if (collect_parts(body, ps) != WL_OK) return 0;
  const Plan P = make_plan(d, ps);
  if (!plan_consistent(d, P)) {
    fail(WL_ERR_INVALID_ARG, "internal: workspace plan and field carving disagree");
    return 0;
  }
  return P.bytes;
}

wl_status wl_sim_create(const wl_sim_desc* desc, const wl_body_desc* body, void* ws, size_t bytes, void* hip_stream,
                        wl_sim** out) {
  if (!out) return fail(WL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  wl_sim_desc d;
  wl_status s = validate_and_default(desc, &d);
  if (s != WL_OK) return s;
  if ((s = validate_body(d, body)) != WL_OK) return s;
  std::vector<wl_body_desc> ps;
  if ((s = collect_parts(body, ps)) != WL_OK) return s;
  Plan P = make_plan(d, ps);
  if (!ws) return fail(WL_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws) & 255u) return fail(WL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < P.bytes) return fail(WL_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than wl_workspace_bytes()");
  if (P.lev[0].elems >= (int64_t(1) << 31)) return fail(WL_ERR_UNSUPPORTED, "grid too large for 32-bit indexing");
  SimBase* impl = make_impl(d.prec, d.ndim);
  impl->desc = d;
  if ((s = collect_parts(body, impl->parts)) != WL_OK) {
    delete impl;
    return s;
  }
  impl->plan = P;
  impl->stream = (hipStream_t)hip_stream;
  if (!carve_any(impl, d, ws, P.bytes)) {
    delete impl;
    return fail(WL_ERR_WORKSPACE_TOO_SMALL, "internal: workspace plan and field carving disagree");
  }
  if (hipGetDevice(&impl->device) != hipSuccess) {
    delete impl;
    return fail(WL_ERR_HIP, "hipGetDevice failed");
  }
  if (hipHostMalloc((void**)&impl->host_pin, kHostPin * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete impl;
    return fail(WL_ERR_HIP, "hipHostMalloc of the read-back buffer failed");
  }

  hipError_t he = hipMemsetAsync(ws, 0, P.bytes, impl->stream);
  if (he != hipSuccess) {
    (void)hipHostFree(impl->host_pin);
    delete impl;
    return fail(WL_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(he));
  }
  s = impl->init();
  if (s != WL_OK) {
    (void)hipHostFree(impl->host_pin);
    delete impl;
    return s;
  }
  wl_sim* h = new wl_sim{impl};
  *out = h;
  return WL_OK;
}

wl_status wl_sim_destroy(wl_sim* sim) {
  if (!sim) return fail(WL_ERR_INVALID_ARG, "sim is NULL");
  if (sim->impl) {
    if (sim->impl->stream) (void)hipStreamSynchronize(sim->impl->stream);
    else (void)hipDeviceSynchronize();
    if (sim->impl->host_pin) (void)hipHostFree(sim->impl->host_pin);
    delete sim->impl;
  }
  delete sim;
  return WL_OK;
}

#define WL_SIM_CHECK(sim) \
  if (!(sim) || !(sim)->impl) return fail(WL_ERR_INVALID_ARG, "sim is NULL")

wl_status wl_measure_body(wl_sim* sim, double t) {
  WL_SIM_CHECK(sim);
  if (!std::isfinite(t)) return fail(WL_ERR_INVALID_ARG, "t must be finite");
  return sim->impl->measure(t);
}

wl_status wl_step(wl_sim* sim, int remeasure, wl_step_stats* stats) {
  WL_SIM_CHECK(sim);
  return sim->impl->step(remeasure, stats);
}

wl_status wl_apply_bc(wl_sim* sim) {
  WL_SIM_CHECK(sim);
  return sim->impl->apply_bc_cur();
}

wl_status wl_conv_diff(wl_sim* sim) {
  WL_SIM_CHECK(sim);
  return sim->impl->conv_diff();
}

wl_status wl_project(wl_sim* sim, double w, wl_solve_stats* stats) {
  WL_SIM_CHECK(sim);
  if (!(w > 0.0) || !std::isfinite(w)) return fail(WL_ERR_INVALID_ARG, "w must be > 0");
  return sim->impl->project_cur(w, stats);
}

wl_status wl_poisson_solve(wl_sim* sim, const void* rhs, void* x_inout, double tol, int itmax,
                           wl_solve_stats* stats) {
  WL_SIM_CHECK(sim);
  if (!std::isfinite(tol)) return fail(WL_ERR_INVALID_ARG, "tol must be finite");
  return sim->impl->poisson(rhs, x_inout, tol, itmax, stats);
}

wl_status wl_forces(wl_sim* sim, double f_pressure[3], double f_viscous[3]) {
  WL_SIM_CHECK(sim);
  if (!f_pressure || !f_viscous) return fail(WL_ERR_INVALID_ARG, "force outputs are NULL");
  return sim->impl->forces(f_pressure, f_viscous);
}

wl_status wl_forces_static(wl_sim* sim, double f_pressure[3], double f_viscous[3]) {
  WL_SIM_CHECK(sim);
  if (!f_pressure || !f_viscous) return fail(WL_ERR_INVALID_ARG, "force outputs are NULL");
  // the sim's GPU is made current for the lookup and the launches, then restored
  int cur = 0;
  WL_HIP(hipGetDevice(&cur));
  const int dev = sim->impl->device;
  if (cur != dev) WL_HIP(hipSetDevice(dev));
  double* scr = nullptr;
  wl_status s = scratch_address(dev, &scr);
  if (s == WL_OK) s = sim->impl->forces_static(scr, f_pressure, f_viscous);
  if (cur != dev) (void)hipSetDevice(cur);
  return s;
}

wl_status wl_field(wl_sim* sim, int which, int level, void** dev_ptr, int64_t shape[4], int64_t strides[4]) {
  WL_SIM_CHECK(sim);
  if (!dev_ptr || !shape || !strides) return fail(WL_ERR_INVALID_ARG, "outputs are NULL");
  return sim->impl->field(which, level, dev_ptr, shape, strides);
}

wl_status wl_levels(wl_sim* sim, int* nlevels, int level, int64_t n_out[3]) {
  WL_SIM_CHECK(sim);
  const Plan& P = sim->impl->plan;
  if (nlevels) *nlevels = P.nlev;
  if (n_out) {
    if (level < 0 || level >= P.nlev) return fail(WL_ERR_INVALID_ARG, "level out of range");
    for (int a = 0; a < 3; ++a) n_out[a] = P.lev[level].n[a];
  }
  return WL_OK;
}

wl_status wl_set_time(wl_sim* sim, double t, double dt_next) {
  WL_SIM_CHECK(sim);
  if (!std::isfinite(t) || !(dt_next > 0.0) || !std::isfinite(dt_next))
    return fail(WL_ERR_INVALID_ARG, "t must be finite and dt_next > 0");
  sim->impl->t = t;
  sim->impl->dt = dt_next;
  return WL_OK;
}

wl_status wl_get_time(wl_sim* sim, double* t, double* dt_next) {
  WL_SIM_CHECK(sim);
  if (t) *t = sim->impl->t;
  if (dt_next) *dt_next = sim->impl->dt;
  return WL_OK;
}

wl_status wl_sim_time(wl_sim* sim, double* t_star) {
  WL_SIM_CHECK(sim);
  if (!t_star) return fail(WL_ERR_INVALID_ARG, "t_star is NULL");
  const wl_sim_desc& d = sim->impl->desc;
  double u = std::sqrt(d.U[0] * d.U[0] + d.U[1] * d.U[1] + d.U[2] * d.U[2]);
  if (u == 0.0) u = 1.0;
  *t_star = sim->impl->t * u / d.L;
  return WL_OK;
}

wl_status wl_profile(wl_sim* sim, int enable) {
  WL_SIM_CHECK(sim);
  return sim->impl->profile(enable ? ~0u : 0u);
}

wl_status wl_profile_groups(wl_sim* sim, uint32_t groups) {
  WL_SIM_CHECK(sim);
  return sim->impl->profile(groups);
}

wl_status wl_profile_read(wl_sim* sim, int kernel, double* total_ms, int64_t* launches) {
  WL_SIM_CHECK(sim);
  return sim->impl->profile_read(kernel, total_ms, launches);
}

wl_status wl_pg_set_weights(wl_sim* sim, const float* host_params) {
  WL_SIM_CHECK(sim);
  return sim->impl->pg_set_weights(host_params);
}

wl_status wl_pg_get_weights(wl_sim* sim, float* host_params) {
  WL_SIM_CHECK(sim);
  return sim->impl->pg_get_weights(host_params);
}

wl_status wl_pg_mode(wl_sim* sim, int mode, double lr, int train_iters, int crops, uint64_t seed) {
  WL_SIM_CHECK(sim);
  return sim->impl->pg_set_mode(mode, lr, train_iters, crops, seed);
}

wl_status wl_pg_forward(wl_sim* sim, const void* x_box, const int64_t n[3], float* y_out) {
  WL_SIM_CHECK(sim);
  return sim->impl->pg_forward(x_box, n, y_out);
}

wl_status wl_pg_train_step(wl_sim* sim, const void* x_box, const float* target, const unsigned char* mask,
                           const int64_t n[3], float* grad_out, double* loss, int apply) {
  WL_SIM_CHECK(sim);
  return sim->impl->pg_train(x_box, target, mask, n, grad_out, loss, apply);
}

wl_status wl_body_update(wl_sim* sim, const wl_body_desc* body) {
  WL_SIM_CHECK(sim);
  return sim->impl->body_update(body);
}

wl_status wl_body_box(wl_sim* sim, int level, int lo[3], int hi[3]) {
  WL_SIM_CHECK(sim);
  if (!lo || !hi) return fail(WL_ERR_INVALID_ARG, "lo/hi are NULL");
  return sim->impl->body_box_of(level, lo, hi);
}

wl_status wl_adj_reset(wl_sim* sim) {
  WL_SIM_CHECK(sim);
  return sim->impl->adj_reset();
}

wl_status wl_adj_forces(wl_sim* sim, const double dir[3], double weight, double* value) {
  WL_SIM_CHECK(sim);
  return sim->impl->adj_forces(dir, weight, value);
}

wl_status wl_adj_step(wl_sim* sim, double tol, wl_step_stats* forward_stats, wl_solve_stats adjoint_stats[2]) {
  WL_SIM_CHECK(sim);
  if (!(tol >= 0.0)) return fail(WL_ERR_INVALID_ARG, "tol must be >= 0");
  return sim->impl->adj_step(tol, forward_stats, adjoint_stats);
}

wl_status wl_adj_step_cfl(wl_sim* sim, double tol, int dt_from_cfl, double* dt_bar, wl_step_stats* forward_stats,
                          wl_solve_stats adjoint_stats[2]) {
  WL_SIM_CHECK(sim);
  if (!(tol >= 0.0)) return fail(WL_ERR_INVALID_ARG, "tol must be >= 0");
  return sim->impl->adj_step_cfl(tol, dt_from_cfl, dt_bar, forward_stats, adjoint_stats);
}

wl_status wl_adj_body_grad(wl_sim* sim, double* dJ_dradius, double* dJ_dspin) {
  WL_SIM_CHECK(sim);
  return sim->impl->adj_body_grad(dJ_dradius, dJ_dspin);
}

wl_status wl_pg_stats(wl_sim* sim, double* last_loss, int64_t* train_steps, int64_t* snapshots,
                      int64_t* guesses_used, int64_t* guesses_tried) {
  WL_SIM_CHECK(sim);
  return sim->impl->pg_stats(last_loss, train_steps, snapshots, guesses_used, guesses_tried);
}

const char* wl_last_error(void) { return g_err.c_str(); }

}  // extern "C"

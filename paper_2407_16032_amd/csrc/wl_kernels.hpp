// HIP kernels of the BDIM projection step (gfx950).  Each kernel cites the
// part of the method it computes; the discrete formulas are documented in
// include/wlmi.h.  Three forms share the arithmetic: generic grid-stride
// kernels (kBlock threads, at most kMaxBlocks blocks, so that per-block partial
// sums fit the reduction slots), z-marching tiles for the large 3-D levels, and
// flat one-vector-per-thread kernels, whose many blocks leave their partials
// in a separate area that a two-stage sum reduces.
#pragma once
#include <type_traits>

#include "wl_device.hpp"

namespace wl {

// tile of the z-marching stencil kernels: 64 x 8 columns, 32 planes deep
#ifndef WL_TY
#define WL_TY 8
#endif
#ifndef WL_TZ
#define WL_TZ 32
#endif
constexpr int kTX = 64, kTY = WL_TY, kTZ = WL_TZ, kTileThreads = kTX * kTY;
// planes between the issue of a marching tile's loads and their use
#ifndef WL_PCG_PF
#define WL_PCG_PF 2
#endif
constexpr int kPF = WL_PCG_PF;
constexpr int kTileMinZ = 8;       // shortest march of a level's tiles
constexpr int kTileTarget = 1024;  // tiles wanted per level (4 per compute unit)
static_assert(kPF >= 2, "pass B consumes two planes per step");

// ---------------------------------------------------------------------------
// bodies (the paper's AutoBody): up to kMaxParts parts, each a shape in its own
// body frame seen through a map x_b = S * Rot(-theta) (x - P) + po, combined
// by signed-distance arithmetic
// ---------------------------------------------------------------------------
constexpr int kMaxParts = 4;
enum { kShapeNone = 0, kShapeSphere = 1, kShapeBox = 2, kShapeGrid = 3, kShapePlane = 4 };
enum { kOpUnion = 0, kOpIntersect = 1, kOpSubtract = 2 };

// signed distance sampled on a grid in the body frame, widened to FP64 in the
// workspace: samples, their central-difference gradients (D arrays) and an
// optional sampled velocity (D arrays or null), x fastest
struct GridSdf {
  const double* s;
  const double* gr;
  const double* v;
  int n[3];
  double o[3], h;
};
struct PartP {
  int kind, op;
  double R;       // sphere radius, plane offset
  double h[3];    // box half extents
  double po[3];   // pivot offset
  double nrm[3];  // plane normal (unit)
  double shell;   // > 0: hollow part
  GridSdf gs;
};
struct BodyP {
  int nparts;   // 0: no body
  int general;  // 0: one rigid part, evaluated by the direct formulas
  PartP p[kMaxParts];
};
struct PartMotion {  // evaluated on the host at time t
  double P[3];       // pivot position
  double ct, st;     // cos/sin of the rotation angle
  double cdot[3];    // velocity of the pivot
  double omega;      // angular velocity about e_z
  double S[3];       // map scale and its rate
  double Sdot[3];
};
struct Motion {
  PartMotion m[kMaxParts];
};

// Cell of the sample grid holding body-frame point xb: lower sample index and
// fractions along each axis; false outside the sampled box.
template <int D>
__host__ __device__ inline bool grid_cell(const GridSdf& G, const double xb[3], int i0[3], double fr[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double u = (xb[a] - G.o[a]) / G.h;
    if (!(u >= 0.0 && u <= double(G.n[a] - 1))) return false;
    int i = (int)floor(u);
    if (i > G.n[a] - 2) i = G.n[a] - 2;
    i0[a] = i;
    fr[a] = u - double(i);
  }
  return true;
}

// Multilinear interpolant of a sample array at the cell found by grid_cell
// (corners in the order of their bit patterns, weights multiplied axis by axis).
template <int D>
__host__ __device__ inline double grid_interp(const GridSdf& G, const double* a, const int i0[3], const double fr[3]) {
#pragma clang fp contract(off)
  double out = 0.0;
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    double w = 1.0;
    int idx = 0, str = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int bit = (c >> k) & 1;
      w = w * (bit ? fr[k] : 1.0 - fr[k]);
      idx += (i0[k] + bit) * str;
      str *= G.n[k];
    }
    out = out + w * a[idx];
  }
  return out;
}

// Signed distance, unit gradient (body frame) and sampled velocity of a part's
// shape at body-frame point xb (before hollowing).
template <int D>
__host__ __device__ inline void shape_eval(const PartP& b, const double xb[3], double& d, double nb[3], double Vs[3]) {
#pragma clang fp contract(off)
  nb[0] = nb[1] = nb[2] = 0.0;
  Vs[0] = Vs[1] = Vs[2] = 0.0;
  if (b.kind == kShapeSphere) {
    double r2 = xb[0] * xb[0] + xb[1] * xb[1];
    if (D == 3) r2 = r2 + xb[2] * xb[2];
    const double r = sqrt(r2);
    d = r - b.R;
    if (r > 0.0) {
      for (int k = 0; k < D; ++k) nb[k] = xb[k] / r;
    } else {
      nb[0] = 1.0;
    }
  } else if (b.kind == kShapeBox) {
    double q[3], o[3];
    for (int k = 0; k < D; ++k) {
      q[k] = fabs(xb[k]) - b.h[k];
      o[k] = fmax(q[k], 0.0);
    }
    double ol2 = o[0] * o[0] + o[1] * o[1];
    if (D == 3) ol2 = ol2 + o[2] * o[2];
    const double olen = sqrt(ol2);
    double qmax = q[0];
    int arg = 0;
    for (int k = 1; k < D; ++k) {
      qmax = fmax(qmax, q[k]);
      if (q[k] > q[arg]) arg = k;
    }
    d = olen + fmin(qmax, 0.0);
    for (int k = 0; k < D; ++k) {
      const double sg = xb[k] >= 0.0 ? 1.0 : -1.0;
      nb[k] = (olen > 0.0) ? sg * o[k] / olen : (k == arg ? sg : 0.0);
    }
  } else if (b.kind == kShapePlane) {
    double s = b.nrm[0] * xb[0] + b.nrm[1] * xb[1];
    if (D == 3) s = s + b.nrm[2] * xb[2];
    d = s - b.R;
    for (int k = 0; k < D; ++k) nb[k] = b.nrm[k];
  } else {  // sampled
    int i0[3] = {0, 0, 0};
    double fr[3] = {0.0, 0.0, 0.0};
    if (!grid_cell<D>(b.gs, xb, i0, fr)) {
      d = 1e300;  // fluid, beyond the kernel's reach
      nb[0] = 1.0;
      return;
    }
    const int cnt = b.gs.n[0] * b.gs.n[1] * (D == 3 ? b.gs.n[2] : 1);
    d = grid_interp<D>(b.gs, b.gs.s, i0, fr);
    double gn[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < D; ++k) gn[k] = grid_interp<D>(b.gs, b.gs.gr + (size_t)k * cnt, i0, fr);
    double m2 = gn[0] * gn[0] + gn[1] * gn[1];
    if (D == 3) m2 = m2 + gn[2] * gn[2];
    const double mag = sqrt(m2);
    if (mag > 0.0) {
      for (int k = 0; k < D; ++k) nb[k] = gn[k] / mag;
    } else {
      nb[0] = 1.0;
    }
    if (b.gs.v)
      for (int k = 0; k < D; ++k) Vs[k] = grid_interp<D>(b.gs, b.gs.v + (size_t)k * cnt, i0, fr);
  }
}

// One rigid part by the direct formulas: d = SDF(x_b), n = Rot(theta) n_b,
// V = dP/dt + omega e_z x (x - P) (+ sampled velocity).
template <int D>
__host__ __device__ inline void part_rigid(const PartP& b, const PartMotion& m, const double x[3], double& d, double n[3],
                                  double V[3]) {
#pragma clang fp contract(off)
  const double rx = x[0] - m.P[0], ry = x[1] - m.P[1], rz = (D == 3) ? x[2] - m.P[2] : 0.0;
  double xb[3];
  xb[0] = m.ct * rx + m.st * ry + b.po[0];
  xb[1] = -m.st * rx + m.ct * ry + b.po[1];
  xb[2] = (D == 3) ? rz + b.po[2] : 0.0;
  double nb[3], Vs[3];
  shape_eval<D>(b, xb, d, nb, Vs);
  n[0] = m.ct * nb[0] - m.st * nb[1];
  n[1] = m.st * nb[0] + m.ct * nb[1];
  n[2] = nb[2];
  V[0] = m.cdot[0] - m.omega * ry + Vs[0];
  V[1] = m.cdot[1] + m.omega * rx + Vs[1];
  V[2] = m.cdot[2] + Vs[2];
}

// One part through its general map.  With J = dx_b/dx = diag(S) Rot(-theta) and
// n_b the shape's unit gradient: g = J^T n_b = Rot(theta)(S n_b), n = g/|g|,
// d = SDF/|g|; V = -J^{-1} dx_b/dt = dP/dt + omega e_z x r - Rot(theta)((S'/S) a)
// with r = x - P and a = Rot(-theta) r.
template <int D>
__host__ __device__ inline void part_general(const PartP& b, const PartMotion& m, const double x[3], double& d, double n[3],
                                    double V[3]) {
#pragma clang fp contract(off)
  const double r0 = x[0] - m.P[0], r1 = x[1] - m.P[1], r2 = (D == 3) ? x[2] - m.P[2] : 0.0;
  const double a0 = m.ct * r0 + m.st * r1, a1 = -m.st * r0 + m.ct * r1, a2 = r2;
  double xb[3];
  xb[0] = m.S[0] * a0 + b.po[0];
  xb[1] = m.S[1] * a1 + b.po[1];
  xb[2] = (D == 3) ? m.S[2] * a2 + b.po[2] : 0.0;
  double dt, nb[3], Vs[3];
  shape_eval<D>(b, xb, dt, nb, Vs);
  if (b.shell > 0.0) {
    const double sg = dt < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) nb[k] = sg * nb[k];
    dt = fabs(dt) - b.shell;
  }
  const double s0 = m.S[0] * nb[0], s1 = m.S[1] * nb[1], s2 = (D == 3) ? m.S[2] * nb[2] : 0.0;
  const double g0 = m.ct * s0 - m.st * s1, g1 = m.st * s0 + m.ct * s1, g2 = s2;
  double gm2 = g0 * g0 + g1 * g1;
  if (D == 3) gm2 = gm2 + g2 * g2;
  const double gm = sqrt(gm2);
  if (gm > 0.0) {
    d = dt / gm;
    n[0] = g0 / gm;
    n[1] = g1 / gm;
    n[2] = g2 / gm;
  } else {
    d = dt;
    n[0] = 1.0;
    n[1] = n[2] = 0.0;
  }
  const double w0 = m.Sdot[0] / m.S[0] * a0, w1 = m.Sdot[1] / m.S[1] * a1,
               w2 = (D == 3) ? m.Sdot[2] / m.S[2] * a2 : 0.0;
  V[0] = m.cdot[0] - m.omega * r1 - (m.ct * w0 - m.st * w1) + Vs[0];
  V[1] = m.cdot[1] + m.omega * r0 - (m.st * w0 + m.ct * w1) + Vs[1];
  V[2] = (D == 3) ? m.cdot[2] - w2 + Vs[2] : 0.0;
}

// signed distance, unit normal and body velocity at point x (FP64).
template <int D>
__host__ __device__ inline void body_eval(const BodyP& b, const Motion& m, const double x[3], double& d, double n[3],
                                 double V[3]) {
  if (!b.general) {
    part_rigid<D>(b.p[0], m.m[0], x, d, n, V);
    return;
  }
  part_general<D>(b.p[0], m.m[0], x, d, n, V);
  for (int k = 1; k < b.nparts; ++k) {
    double db, nb[3], Vb[3];
    part_general<D>(b.p[k], m.m[k], x, db, nb, Vb);
    // a subtracted part enters with d and n negated (a product with -1: the
    // three-way branch on op, with the negation inside it, was compiled for
    // gfx950 into a flow that skipped the negation)
    const int op = b.p[k].op;
    const double sg = (op == kOpSubtract) ? -1.0 : 1.0;
    db = sg * db;
    for (int j = 0; j < 3; ++j) nb[j] = sg * nb[j];
    const bool take = (op == kOpUnion) ? (db < d) : (db > d);
    if (take) {
      d = db;
      for (int j = 0; j < 3; ++j) {
        n[j] = nb[j];
        V[j] = Vb[j];
      }
    }
  }
}

// Sample gradients of a gridded SDF by central differences (one-sided on the
// grid's faces), FP64: gr[k][i] = (s[i + e_k] - s[i - e_k]) / (2h).
template <int D>
__global__ void __launch_bounds__(kBlock) k_grid_grad(const double* s, double* gr, int n0, int n1, int n2, double h) {
#pragma clang fp contract(off)
  const int n[3] = {n0, n1, D == 3 ? n2 : 1};
  const int cnt = n[0] * n[1] * n[2];
  const int str[3] = {1, n[0], n[0] * n[1]};
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < cnt; lin += gridDim.x * kBlock) {
    const int I[3] = {lin % n[0], (lin / n[0]) % n[1], lin / (n[0] * n[1])};
    for (int k = 0; k < D; ++k) {
      double gk;
      if (I[k] == 0) gk = (s[lin + str[k]] - s[lin]) / h;
      else if (I[k] == n[k] - 1) gk = (s[lin] - s[lin - str[k]]) / h;
      else gk = (s[lin + str[k]] - s[lin - str[k]]) / (2.0 * h);
      gr[(size_t)k * cnt + lin] = gk;
    }
  }
}

// widen caller samples of the simulation's precision to FP64
template <typename T>
__global__ void __launch_bounds__(kBlock) k_widen(const T* src, double* dst, int64_t cnt) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * kBlock)
    dst[i] = double(src[i]);
}

// Moments of the kernel; beyond its support (|s| >= 1) they are the full integrals,
// exactly 0 / 1 for mu0 and 0 for mu1 (the closed forms would leave sin(pi) rounding).
__device__ inline double kern_mu0(double d, double eps) {
#pragma clang fp contract(off)
  const double s = d / eps;
  if (s >= 1.0) return 1.0;
  if (s <= -1.0) return 0.0;
  return 0.5 * (1.0 + s) + sin(M_PI * s) / (2.0 * M_PI);
}
__device__ inline double kern_mu1(double d, double eps) {
#pragma clang fp contract(off)
  const double s = d / eps;
  if (fabs(s) >= 1.0) return 0.0;
  return eps * (0.25 * (1.0 - s * s) - (s * sin(M_PI * s) + (1.0 + cos(M_PI * s)) / M_PI) / (2.0 * M_PI));
}
__device__ inline double kern_K(double d, double eps) {
#pragma clang fp contract(off)
  const double s = d / eps;
  return fabs(s) < 1.0 ? 0.5 * (1.0 + cos(M_PI * s)) / eps : 0.0;
}

constexpr double kMu0Cut = 1e-6;  // faces with mu0 below this are solid

// ---------------------------------------------------------------------------
// Closed-form coefficients away from the body.  Outside a level's body box
// (padded indices, inclusive) measure leaves every coefficient at its body-free
// value: L_a = Lstd on interior faces and 0 on non-periodic boundary faces, iD
// from those L, and on the fine level mu0 = L, mu1 = 0, V = 0.  Kernels whose
// whole stencil lies outside the box evaluate these instead of loading them;
// the values are bit-identical to the stored ones (sums of 0 and a power of two,
// then one correctly rounded division).
// ---------------------------------------------------------------------------
struct StdBox {
  int lo[3], hi[3];  // empty when lo[0] > hi[0]
  double Lstd;       // 1 on the fine level, times 2^(D-2) per coarsening
  // iD of a cell with c non-periodic boundary faces, 1/(-(Lstd (2D - c))), in each
  // precision (the host's correctly rounded division gives the device's value)
  float iDf[4];
  double iDd[4];
};
template <typename T>
__device__ __forceinline__ T std_iD(const StdBox& B, int c);
template <>
__device__ __forceinline__ float std_iD<float>(const StdBox& B, int c) {
  return B.iDf[c];
}
template <>
__device__ __forceinline__ double std_iD<double>(const StdBox& B, int c) {
  return B.iDd[c];
}

// Does the index range [a_k, b_k] per axis (may extend past the padded range) miss
// the box?  On a periodic axis a range that leaves 1..N is taken as the whole axis.
template <int D>
__device__ __forceinline__ bool std_miss(const StdBox& B, const Grid3& g, const int a[3], const int b[3]) {
  if (B.lo[0] > B.hi[0]) return true;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int lo = a[k], hi = b[k];
    if (g.per[k] && (lo < 1 || hi > g.n[k])) {
      lo = 0;
      hi = g.n[k] + 1;
    }
    if (hi < B.lo[k] || lo > B.hi[k]) return true;
  }
  return false;
}

// L_a at face index Ia (1..N_a+1) along a, body-free
template <typename T>
__device__ __forceinline__ T L_std(const Grid3& g, const StdBox& B, int a, int Ia) {
  return (g.per[a] || (Ia >= 2 && Ia <= g.n[a])) ? T(B.Lstd) : T(0);
}

// inverse diagonal of cell (i, j, k), body-free (0 off the interior)
template <typename T, int D>
__device__ __forceinline__ T iD_std(const Grid3& g, const StdBox& B, int i, int j, int k) {
  const int I[3] = {i, j, k};
  int cnt = 2 * D;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (I[a] < 1 || I[a] > g.n[a]) return T(0);
    if (!g.per[a]) cnt -= (I[a] == 1 ? 1 : 0) + (I[a] == g.n[a] ? 1 : 0);
  }
  return T(1) / (-(T(B.Lstd) * T(cnt)));
}

// Closed-form inverse diagonals by the number of non-periodic boundary faces of
// a cell (0..3), computed once per thread (same expression as iD_std).
template <typename T, int D>
struct StdDiag {
  T v[4];
  __device__ explicit StdDiag(const StdBox& B) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = std_iD<T>(B, c);
  }
  __device__ __forceinline__ T at(const Grid3& g, int i, int j, int k) const {
    const int I[3] = {i, j, k};
    int nb = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (I[a] < 1 || I[a] > g.n[a]) return T(0);
      if (!g.per[a]) nb += (I[a] == 1 ? 1 : 0) + (I[a] == g.n[a] ? 1 : 0);
    }
    return v[nb];
  }
};

// is the cube [I - m, I + m] outside the box?
template <int D>
__device__ __forceinline__ bool std_point(const StdBox& B, const Grid3& g, const int I[3], int m) {
  const int a[3] = {I[0] - m, I[1] - m, I[2] - m}, b[3] = {I[0] + m, I[1] + m, I[2] + m};
  return std_miss<D>(B, g, a, b);
}

// measure!: mu0 (= fine Poisson L, 0 on non-periodic boundary faces), mu1 = mu1(d) n, V.
// blockIdx.y = component.
// Points outside the box [lo, hi] (padded coordinates) keep their previous values:
// the caller guarantees they lie outside the body's reach at both the previous and
// the current measure time.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_measure(Grid3 g, BodyP b, Motion m, double eps,
                                                    Vec3<T> mu0, Vec9<T> mu1, Vec3<T> V, int3 lo, int3 hi) {
  const int c = blockIdx.y;
  const int P0 = hi.x - lo.x + 1, P1 = hi.y - lo.y + 1, P2 = (D == 3) ? hi.z - lo.z + 1 : 1;
  const int total = P0 * P1 * P2;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I0 = lo.x + lin % P0, t = lin / P0, I1 = lo.y + t % P1, I2 = (D == 3) ? lo.z + t / P1 : 0;
    const int I[3] = {I0, I1, I2};
    const int idx = I0 + I1 * g.s[1] + I2 * g.s[2];
    double m0 = 1.0, m1 = 0.0, vb[3] = {0.0, 0.0, 0.0}, nn[3] = {0.0, 0.0, 0.0}, d = 1e300;
    if (b.nparts != 0) {
      double x[3];
      for (int a = 0; a < 3; ++a) x[a] = (a == c) ? I[a] - 1.0 : I[a] - 0.5;
      body_eval<D>(b, m, x, d, nn, vb);
      m0 = kern_mu0(d, eps);
      m1 = kern_mu1(d, eps);
      if (m0 < kMu0Cut) {
        m0 = 0.0;
        m1 = 0.0;
      }
    }
    const bool bnd = !g.per[c] && (I[c] <= 1 || I[c] == g.n[c] + 1);
    mu0.c[c][idx] = bnd ? T(0) : T(m0);
    if (b.nparts != 0) {
      for (int j = 0; j < D; ++j) mu1.c[c * D + j][idx] = T(m1 * nn[j]);
      V.c[c][idx] = (d < 2.0 + eps) ? T(vb[c]) : T(0);
    }
  }
}

// ---------------------------------------------------------------------------
// multigrid coefficients: inverse diagonal and coefficient restriction
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_inv_diag(Grid3 g, Vec3<T> L, T* iD, int3 lo, int3 hi) {
  // the cells lo..hi (interior indices, inclusive) only
  const int m0 = hi.x - lo.x + 1, m1 = hi.y - lo.y + 1, m2 = (D == 3) ? hi.z - lo.z + 1 : 1;
  const int total = m0 * m1 * m2;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I0 = lin % m0 + lo.x, t = lin / m0, I1 = t % m1 + lo.y, I2 = (D == 3) ? t / m1 + lo.z : 0;
    const int I[3] = {I0, I1, I2};
    const int idx = I0 + I1 * g.s[1] + I2 * g.s[2];
    T Dg = T(0);
    for (int a = 0; a < D; ++a) {
      const int off = (g.per[a] && I[a] == g.n[a]) ? -(g.n[a] - 1) * g.s[a] : g.s[a];
      Dg = Dg - (L.c[a][idx] + L.c[a][idx + off]);
    }
    iD[idx] = (Dg != T(0)) ? T(1) / Dg : T(0);
  }
}

// L_c,a[J] = 1/2 * sum of the fine a-faces covering the coarse a-face.  blockIdx.y = a.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_restrict_L(Grid3 f, Grid3 c, Vec3<T> Lf, Vec3<T> Lc, int3 lo, int3 hi) {
  const int a = blockIdx.y;
  // coarse faces: J_a in 1..Nc_a+1, other axes 1..Nc, within lo..hi
  const int l3[3] = {lo.x, lo.y, lo.z}, h3[3] = {hi.x, hi.y, hi.z};
  int st[3], m[3];
  for (int k = 0; k < 3; ++k) {
    const int top = (k < D) ? (c.n[k] + (k == a ? 1 : 0)) : 1;
    st[k] = (k < D) ? max(1, l3[k]) : 0;
    m[k] = (k < D) ? max(0, min(top, h3[k]) - st[k] + 1) : 1;
  }
  const int total = m[0] * m[1] * m[2];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int J0 = lin % m[0] + st[0], t = lin / m[0], J1 = t % m[1] + st[1], J2 = (D == 3) ? t / m[1] + st[2] : 0;
    const int J[3] = {J0, J1, J2};
    int base = 0;
    for (int k = 0; k < D; ++k) base += (2 * J[k] - 1) * f.s[k];
    // pair sums along the remaining axes, in axis order
    const int b0 = (a == 0) ? 1 : 0, b1 = (a == 2) ? 1 : 2;  // the other axes (D==3)
    T v;
    if (D == 2) {
      const int o = (a == 0) ? f.s[1] : f.s[0];
      v = Lf.c[a][base] + Lf.c[a][base + o];
    } else {
      const int ob0 = f.s[b0], ob1 = f.s[b1];
      v = (Lf.c[a][base] + Lf.c[a][base + ob0]) + (Lf.c[a][base + ob1] + Lf.c[a][base + ob0 + ob1]);
    }
    const int cidx = J0 + J1 * c.s[1] + J2 * c.s[2];
    Lc.c[a][cidx] = T(0.5) * v;
  }
}

// ---------------------------------------------------------------------------
// convection-diffusion flux and f~ = u0 + dt R(u) - V
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ int lin3(const Grid3& g, int a, int b, int c) {
  return a + b * g.s[1] + ((D == 3) ? c * g.s[2] : 0);
}

// Flux Phi_cj at the (wrapped) index J.
template <typename T, int D>
__device__ __forceinline__ T phi_cj(const Grid3& g, const Vec3<T>& u, int c, int j, const int J[3], T nu) {
  int Jc[3] = {J[0], J[1], J[2]};
  Jc[c] = wrapc(J[c] - 1, c, g);
  int Jj[3] = {J[0], J[1], J[2]};
  Jj[j] = wrapc(J[j] - 1, j, g);
  const int iJ = lin3<T, D>(g, J[0], J[1], J[2]);
  const T a = T(0.5) * (u.c[j][iJ] + u.c[j][lin3<T, D>(g, Jc[0], Jc[1], Jc[2])]);
  const T uc = u.c[c][iJ];
  const T m1 = u.c[c][lin3<T, D>(g, Jj[0], Jj[1], Jj[2])];
  const bool up = a >= T(0);
  int F[3] = {J[0], J[1], J[2]};
  const int fx = up ? J[j] - 2 : J[j] + 1;
  bool ok;
  if (g.per[j]) {
    F[j] = wrapc(fx, j, g);
    ok = true;
  } else {
    F[j] = fx;
    ok = fx >= 1 && fx <= (j == c ? g.n[j] + 1 : g.n[j]);
  }
  T Q;
  if (ok) {
    const T far = u.c[c][lin3<T, D>(g, F[0], F[1], F[2])];
    Q = up ? quick_lim(far, m1, uc) : quick_lim(far, uc, m1);
  } else {
    Q = T(0.5) * (uc + m1);
  }
  return a * Q - nu * (uc - m1);
}

template <typename T, int D>
__device__ __forceinline__ T resid_c(const Grid3& g, const Vec3<T>& u, int c, const int I[3], T nu) {
  T acc = T(0);
  for (int j = 0; j < D; ++j) {
    int Jp[3] = {I[0], I[1], I[2]};
    Jp[j] = wrapc(I[j] + 1, j, g);
    acc = acc + (phi_cj<T, D>(g, u, c, j, I, nu) - phi_cj<T, D>(g, u, c, j, Jp, nu));
  }
  return acc;
}

// Same flux with plain offsets, valid when every +-2 stencil point is interior.
template <typename T, int D>
__device__ __forceinline__ T phi_fast(const Vec3<T>& u, int c, int j, int id, int sc, int sj, T nu) {
  const T a = T(0.5) * (u.c[j][id] + u.c[j][id - sc]);
  const T uc = u.c[c][id];
  const T m1 = u.c[c][id - sj];
  const bool up = a >= T(0);
  const T far = up ? u.c[c][id - 2 * sj] : u.c[c][id + sj];
  const T Q = up ? quick_lim(far, m1, uc) : quick_lim(far, uc, m1);
  return a * Q - nu * (uc - m1);
}

template <typename T, int D>
__device__ __forceinline__ T resid_fast(const Grid3& g, const Vec3<T>& u, int c, int id, T nu) {
  const int sc = g.s[c];
  T acc = T(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int sj = g.s[j];
    acc = acc + (phi_fast<T, D>(u, c, j, id, sc, sj, nu) - phi_fast<T, D>(u, c, j, id + sj, sc, sj, nu));
  }
  return acc;
}

// f~_c = u0_c + dt R_c(u) - V_c at padded face I (R = 0 off the unknown faces).
// mode 0: f~ (with body velocity if has_body); mode 1: f = R only.
template <typename T, int D>
__device__ __forceinline__ void flux_face(const Grid3& g, const Vec3<T>& u, const Vec3<T>& u0, const Vec3<T>& V,
                                          const Vec3<T>& f, T dt, T nu, int has_body, int mode, const StdBox& B,
                                          int c, const int I[3]) {
  const int idx = lin3<T, D>(g, I[0], I[1], I[2]);
  bool unknown = true;
  for (int a = 0; a < D; ++a) {
    const int lo = (a == c && !g.per[a]) ? 2 : 1;
    unknown = unknown && I[a] >= lo && I[a] <= g.n[a];
  }
  // the point-wise loads go first, so they overlap the stencil's
  const bool needV = mode == 0 && has_body && !std_point<D>(B, g, I, 0);  // V = 0 outside the box
  const T vb = needV ? V.c[c][idx] : T(0);
  const T u0v = (mode == 0) ? u0.c[c][idx] : T(0);
  T R = T(0);
  if (unknown) {
    // interior fast path: the +-2 stencil needs no wrap and every far point is valid
    bool fast = true;
    for (int a = 0; a < D; ++a) fast = fast && I[a] >= 3 && I[a] <= g.n[a] - 2;
    R = fast ? resid_fast<T, D>(g, u, c, idx, nu) : resid_c<T, D>(g, u, c, I, nu);
  }
  if (mode == 1) {
    f.c[c][idx] = R;
  } else {
    T v = u0v + dt * R;
    if (needV) v = v - vb;
    f.c[c][idx] = v;
  }
}

// Every padded face, grid-stride (2-D, and the residual-only mode).  blockIdx.y = c.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_flux(Grid3 g, Vec3<T> u, Vec3<T> u0, Vec3<T> V,
                                                 Vec3<T> f, T dt, T nu, int has_body, int mode, StdBox B) {
  const int c = blockIdx.y;
  const int P0 = g.n[0] + 2, P1 = g.n[1] + 2, P2 = (D == 3) ? g.n[2] + 2 : 1;
  const int total = P0 * P1 * P2;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I[3] = {lin % P0, (lin / P0) % P1, (D == 3) ? lin / (P0 * P1) : 0};
    flux_face<T, D>(g, u, u0, V, f, dt, nu, has_body, mode, B, c, I);
  }
}

// 3-D form that shares face fluxes between neighbouring faces: each thread
// marches one column in z and carries phi_cz of the next plane to the next
// step, and its +x flux is the next lane's own phi_cx, so a face costs four flux
// evaluations instead of six.  Lane 63 only supplies that flux, so bricks step
// by 63 columns; a block stacks kRW waves (rows) in y and needs no barrier.
// Faces whose +1 neighbour wraps a periodic axis take the per-face form.
#ifndef WL_RW
#define WL_RW 1
#endif
#ifndef WL_RZ
#define WL_RZ 16
#endif
constexpr int kRX = 64, kRW = WL_RW, kRZ = WL_RZ, kReuseThreads = kRX * kRW;

// the face fluxes an unknown face uses lie at 1..N_j + 1 along j and 1..N_a on
// the other axes; phi_cj reads only valid points there
__device__ __forceinline__ bool phi_needed(const Grid3& g, int j, int p0, int p1, int p2) {
  const int P[3] = {p0, p1, p2};
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) ok = ok && P[a] >= 1 && P[a] <= g.n[a] + (a == j ? 1 : 0);
  return ok;
}

// phi_cj at P (0 where no unknown face uses it): the plain-offset form where no
// point of its stencil wraps or needs the boundary rule, else the general one
// (both compute the same value)
template <typename T>
__device__ __forceinline__ T phi_at(const Grid3& g, const Vec3<T>& u, int c, int j, int p0, int p1, int p2, T nu) {
  if (!phi_needed(g, j, p0, p1, p2)) return T(0);
  const int P[3] = {p0, p1, p2};
  if (P[j] >= 3 && P[j] <= g.n[j] - 1 && P[c] >= 2)
    return phi_fast<T, 3>(u, c, j, lin3<T, 3>(g, p0, p1, p2), g.s[c], g.s[j], nu);
  return phi_cj<T, 3>(g, u, c, j, P, nu);
}

// fm in the lanes whose bit of the wave mask is set, else fp.  In FP32 this is one
// v_cndmask of its own: written as a select the compiler moves each far-point
// load behind the upwind test (into a branch, or as a load from a selected
// address), which costs a second round trip to memory per plane.
template <typename T>
__device__ __forceinline__ T pick_far(bool up, T fm, T fp) {
  return up ? fm : fp;
}
template <>
__device__ __forceinline__ float pick_far<float>(bool up, float fm, float fp) {
  const uint64_t mask = __builtin_amdgcn_ballot_w64(up);
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(fp), "v"(fm), "s"(mask));
  return r;
}

// p, the same in every lane, as a scalar value that the loop optimiser cannot
// turn into per-lane pointers: each load's address is then that scalar base
// plus a lane offset kept for the whole march (one add), instead of a 64-bit
// pointer per field and plane held in vector registers
typedef __attribute__((address_space(1))) char gchar;  // global memory
__device__ __forceinline__ gchar* uniform_ptr(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
  return reinterpret_cast<gchar*>((uint64_t(hi) << 32) | lo);
}

// x's value in the next lane (lane 63 gets an unspecified value): a DPP wave
// shift in FP32, one VALU instruction instead of a permute through the LDS unit
template <typename T>
__device__ __forceinline__ T next_lane(T x) {
  return __shfl_down(x, 1, 64);
}
template <>
__device__ __forceinline__ float next_lane<float>(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130, 0xf, 0xf, false));  // wave_shl:1
}

// phi_fast's flux from values already loaded: a = (a0 + a1)/2, uc and m1 at the
// face and its -j neighbour, fm / fp the far point for a >= 0 / a < 0
template <typename T>
__device__ __forceinline__ T phi_vals(T a0, T a1, T uc, T m1, T fm, T fp, T nu) {
  const T a = T(0.5) * (a0 + a1);
  const bool up = a >= T(0);
  const T far = pick_far<T>(up, fm, fp);
  // one limiter on arguments picked by the upwind test (the same value as the
  // two-sided select of the general form)
  const T Q = quick_lim(far, up ? m1 : uc, up ? uc : m1);
  return a * Q - nu * (uc - m1);
}

// phi_vals with the general form's rules for a face near a non-periodic x
// boundary (its y and z stencil interior): 0 where no unknown face uses the flux
// (need false), the central value where the far point for the upwind side lies
// outside (up_ok / dn_ok false for a >= 0 / a < 0)
template <typename T>
__device__ __forceinline__ T phi_vals_edge(T a0, T a1, T uc, T m1, T fm, T fp, T nu, bool need, bool up_ok,
                                           bool dn_ok) {
  const T a = T(0.5) * (a0 + a1);
  const bool up = a >= T(0);
  const T far = pick_far<T>(up, fm, fp);
  T Q = quick_lim(far, up ? m1 : uc, up ? uc : m1);
  if (!(up ? up_ok : dn_ok)) Q = T(0.5) * (uc + m1);
  const T r = a * Q - nu * (uc - m1);
  return need ? r : T(0);
}

// Is padded index I inside the box [lo, hi] itself (no periodic widening)?
__device__ __forceinline__ bool in_box3(const StdBox& B, const int I[3]) {
  return B.lo[0] <= B.hi[0] && I[0] >= B.lo[0] && I[0] <= B.hi[0] && I[1] >= B.lo[1] && I[1] <= B.hi[1] &&
         I[2] >= B.lo[2] && I[2] <= B.hi[2];
}

// FUSE = 0: f = f~ on every face.  FUSE = 1 (predictor) / 2 (corrector): the BDIM
// blend is applied here to every face outside the body box [lo, hi], where the
// coefficients are body-free (mu0 = L, mu1 = 0, V = 0): uo = L f~, or with the
// corrector uo = (u + L f~)/2, u being this stage's velocity at the same face.
// f~ itself is stored only within one face of the box, for k_bdim_box, which
// blends the faces of the box.  (On a periodic axis the body-free test also counts
// the ghost faces 0 and N+1 as inside; ghost faces are rewritten by the boundary
// conditions straight after the blend, so they take the body-free form here.)
// uo may be u0: each face reads u0 only at its own index, before its store.
// The column march of k_flux_reuse for component C (a compile-time constant, so
// the advecting velocities that coincide with stencil values of u_C are loaded once).
template <typename T, int FUSE, int C>
__device__ __forceinline__ void flux_column(const Grid3& g, const Vec3<T>& u, const Vec3<T>& u0, const Vec3<T>& V,
                                            const Vec3<T>& f, const Vec3<T>& uo, T dt, T nu, int has_body,
                                            const StdBox& B, int lane, int I0, int I1, int z0) {
  constexpr int c = C;
  const int P0 = g.n[0] + 2, P2 = g.n[2] + 2;
  const bool col = lane < kRX - 1 && I0 < P0;
  const int z1 = min(z0 + kRZ, P2);
  T phz = phi_at<T>(g, u, c, 2, I0, I1, z0, nu);
  // u_C at the face and at -1, +1 in z, carried from plane to plane on the fast path
  T cz0 = T(0), cz1 = T(0), cz2 = T(0);
  // fast-path addresses: a base per field and plane, the same for the whole wave,
  // plus one of five 32-bit byte offsets per lane (the column and its +-1, +-2
  // rows in y) and a constant for the x offsets, so that no lane computes a full
  // address per load; the offsets are used only on the fast path (I0, I1 >= 3)
  const int s1 = g.s[1], s2 = g.s[2];
  constexpr int E = int(sizeof(T));
  // (lanes past the row, which store nothing, load at its last column)
  const uint32_t ob = uint32_t(min(I0, P0 - 1) + I1 * s1) * uint32_t(E), sb = uint32_t(s1) * uint32_t(E);
  const uint32_t oy[5] = {ob - 2 * sb, ob - sb, ob, ob + sb, ob + 2 * sb};
  // EDGE planes (the first and last bricks of a row on a non-periodic x axis):
  // which of the lane's fluxes are used (x face; y and z faces), and whether the
  // x face's far point lies inside for a >= 0 and for a < 0
  // (an x-face flux is used on faces 1..N0 + 1 of every component, a y or z one on
  // columns 1..N0; the far point of an x face is inside on 1..N0, or on 1..N0 + 1
  // for u_x)
  const bool need_x = I0 >= 1 && I0 <= g.n[0] + 1, need_o = I0 >= 1 && I0 <= g.n[0];
  const bool up_ok = I0 >= 3, dn_ok = I0 + 1 <= g.n[0] + (c == 0 ? 1 : 0);
  // value at row offset dy (-2..2) and x offset dx of plane I2 + dz of field q
  typedef __attribute__((address_space(1))) T gT;
  auto at = [&](const T* q, int I2, int dz, int dy, int dx) -> T {
    gchar* base = uniform_ptr(q + size_t(I2 + dz) * size_t(s2));
    return *reinterpret_cast<gT*>(base + size_t(oy[dy + 2]) + dx * E);
  };
  auto put_fast = [&](T* q, int I2, T val) {
    *reinterpret_cast<gT*>(uniform_ptr(q + size_t(I2) * size_t(s2)) + size_t(ob)) = val;
  };
  // one plane of the march: MODE 1 (FAST) the plain-offset stencil, every lane
  // of the wave interior enough for it; MODE 2 (EDGE) the same loads with the
  // general form's x-boundary rules per lane (non-periodic x, rows and planes
  // interior); MODE 0 the general form per lane
  auto plane = [&](auto mode_tag, int I2) {
    constexpr int MODE = decltype(mode_tag)::value;
    constexpr bool FAST = MODE == 1, LOADS = MODE != 0;
    T phx, phy, phyn, phzn;
    // u0 at the face (column clamped into the row for the lanes that store nothing)
    // is loaded ahead of the stencil; with FUSE = 2 also u at the face
    const int idx = lin3<T, 3>(g, min(I0, P0 - 1), I1, I2);
    T u0v;
    T uself = T(0);
    if (LOADS) {
      u0v = at(u0.c[c], I2, 0, 0, 0);
      // keeps the load here: the compiler would otherwise sink it into the
      // store block below, after the fluxes, a second round trip per plane
      asm volatile("" ::: "memory");
      // one straight block of loads: every value the four face fluxes can use,
      // both QUICK far points of each included, so no address waits for the
      // upwind test and the whole stencil is one round trip to memory
      const T* q = u.c[c];
      const T zm1 = cz0, c0 = cz1, zp1 = cz2;
      const T xm1 = at(q, I2, 0, 0, -1), xm2 = at(q, I2, 0, 0, -2), xp1 = at(q, I2, 0, 0, 1);
      const T ym1 = at(q, I2, 0, -1, 0), ym2 = at(q, I2, 0, -2, 0), yp1 = at(q, I2, 0, 1, 0),
              yp2 = at(q, I2, 0, 2, 0);
      const T zp2 = at(q, I2, 2, 0, 0);
      cz0 = c0;
      cz1 = zp1;
      cz2 = zp2;
      // the advecting velocities (at the face and at its -C neighbour); those of
      // component C are values of the stencil
      const int cx = C == 0 ? -1 : 0, cy = C == 1 ? -1 : 0, cz = C == 2 ? -1 : 0;
      const T ax0 = C == 0 ? c0 : at(u.c[0], I2, 0, 0, 0), ax1 = C == 0 ? xm1 : at(u.c[0], I2, cz, cy, cx);
      const T ay0 = C == 1 ? c0 : at(u.c[1], I2, 0, 0, 0), ay1 = C == 1 ? ym1 : at(u.c[1], I2, cz, cy, cx);
      const T ayn0 = C == 1 ? yp1 : at(u.c[1], I2, 0, 1, 0), ayn1 = C == 1 ? c0 : at(u.c[1], I2, cz, 1 + cy, cx);
      const T azn0 = C == 2 ? zp1 : at(u.c[2], I2, 1, 0, 0), azn1 = C == 2 ? c0 : at(u.c[2], I2, 1 + cz, cy, cx);
      if (FAST) {
        phx = phi_vals<T>(ax0, ax1, c0, xm1, xm2, xp1, nu);
      } else {
        phx = phi_vals_edge<T>(ax0, ax1, c0, xm1, xm2, xp1, nu, need_x, up_ok, dn_ok);
      }
      phy = phi_vals<T>(ay0, ay1, c0, ym1, ym2, yp1, nu);
      phyn = phi_vals<T>(ayn0, ayn1, yp1, c0, ym1, yp2, nu);
      phzn = phi_vals<T>(azn0, azn1, zp1, c0, zm1, zp2, nu);
      if (!FAST) {
        phy = need_o ? phy : T(0);
        phyn = need_o ? phyn : T(0);
        phzn = need_o ? phzn : T(0);
      }
      if (FUSE == 2) uself = c0;
    } else {
      u0v = u0.c[c][idx];
      phx = phi_at<T>(g, u, c, 0, I0, I1, I2, nu);
      phy = phi_at<T>(g, u, c, 1, I0, I1, I2, nu);
      phyn = phi_at<T>(g, u, c, 1, I0, I1 + 1, I2, nu);
      phzn = phi_at<T>(g, u, c, 2, I0, I1, I2 + 1, nu);
      if (FUSE == 2) uself = u.c[c][idx];
    }
    const T phxn = next_lane<T>(phx);  // every lane of the wave takes part
    if (col) {
      const int I[3] = {I0, I1, I2};
      // on the fast planes every face is an unknown two or more cells from each
      // boundary: no wrap, and L = B.Lstd; on the EDGE planes the same holds in y
      // and z, and x (not periodic) decides
      bool unknown = true, wraps = false;
      if (MODE == 2) {
        unknown = I0 >= (c == 0 ? 2 : 1) && I0 <= g.n[0];
      } else if (MODE == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int lo = (a == c && !g.per[a]) ? 2 : 1;
          unknown = unknown && I[a] >= lo && I[a] <= g.n[a];
          wraps = wraps || (g.per[a] && I[a] == g.n[a]);
        }
      }
      const bool needV = has_body && !std_point<3>(B, g, I, 0);  // V = 0 outside the box
      const T vb = needV ? (LOADS ? at(V.c[c], I2, 0, 0, 0) : V.c[c][idx]) : T(0);
      T R = T(0);
      if (unknown) {
        if (MODE == 0 && wraps) {
          R = resid_c<T, 3>(g, u, c, I, nu);
        } else {
          R = R + (phx - phxn);
          R = R + (phy - phyn);
          R = R + (phz - phzn);
        }
      }
      T v = u0v + dt * R;
      if (needV) v = v - vb;
      auto put = [&](T* q, T val) {
        if (LOADS) put_fast(q, I2, val);
        else q[idx] = val;
      };
      if (FUSE == 0) {
        put(f.c[c], v);
      } else {
        if (has_body && !std_point<3>(B, g, I, 1)) put(f.c[c], v);
        if (!in_box3(B, I)) {
          const T Lf = FAST ? T(B.Lstd) : MODE == 2 ? (c == 0 ? L_std<T>(g, B, 0, I0) : T(B.Lstd))
                                                    : L_std<T>(g, B, c, I[c]);
          T acc = has_body ? Lf * v : v;
          if (FUSE == 2) acc = T(0.5) * (uself + acc);
          put(uo.c[c], acc);
        }
      }
    }
    phz = phzn;
  };
  // planes [za, zb) take the fast or the EDGE path: the march is split into
  // three loops, so that the middle loop's body has no branch whose join would
  // make it wait for u0 before the stencil's loads go out (the two may be in
  // flight together)
  typedef std::integral_constant<int, 0> Gen;
  int za = z0, zb = z0;
  const bool fy = I1 >= 3 && I1 <= g.n[1] - 2;  // the same for the whole wave
  const bool fx = __builtin_amdgcn_ballot_w64(I0 >= 3 && I0 <= g.n[0] - 2) == __builtin_amdgcn_read_exec();
  if (fy && (fx || !g.per[0])) {
    za = min(max(z0, 3), z1);
    zb = max(za, min(z1, g.n[2] - 1));
  }
  for (int I2 = z0; I2 < za; ++I2) plane(Gen{}, I2);
  if (za < zb) {
    cz0 = at(u.c[c], za, -1, 0, 0);
    cz1 = at(u.c[c], za, 0, 0, 0);
    cz2 = at(u.c[c], za, 1, 0, 0);
    if (fx) {
      for (int I2 = za; I2 < zb; ++I2) plane(std::integral_constant<int, 1>{}, I2);
    } else {
      for (int I2 = za; I2 < zb; ++I2) plane(std::integral_constant<int, 2>{}, I2);
    }
  }
  for (int I2 = zb; I2 < z1; ++I2) plane(Gen{}, I2);
}

template <typename T, int FUSE>
__global__ void __launch_bounds__(kReuseThreads) k_flux_reuse(Grid3 g, Vec3<T> u, Vec3<T> u0, Vec3<T> V, Vec3<T> f,
                                                              Vec3<T> uo, T dt, T nu, int has_body, StdBox B,
                                                              int nbx, int nby, int nbz) {
  // one block per brick and component; the XCDs take contiguous ranges of
  // (brick, component) with the component fastest, so the three blocks of a brick
  // run together on one XCD and share the velocity they read through its L2
  const int nb = nbx * nby * nbz * 3;
  const int b = blockIdx.x;
  const int full = (nb / 8) * 8;
  const int tc = (b < full) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int c = tc % 3, t = tc / 3;
  const int bx = t % nbx, r1 = t / nbx, by = r1 % nby, bz = r1 / nby;
  const int lane = (int)threadIdx.x % kRX;
  const int I0 = bx * (kRX - 1) + lane, I1 = by * kRW + (int)threadIdx.x / kRX;
  if (I1 >= g.n[1] + 2) return;  // whole waves: no lane of the wave is needed, and no barrier follows
  const int z0 = bz * kRZ;
  // c is the same for the whole block
  if (c == 0) flux_column<T, FUSE, 0>(g, u, u0, V, f, uo, dt, nu, has_body, B, lane, I0, I1, z0);
  else if (c == 1) flux_column<T, FUSE, 1>(g, u, u0, V, f, uo, dt, nu, has_body, B, lane, I0, I1, z0);
  else flux_column<T, FUSE, 2>(g, u, u0, V, f, uo, dt, nu, has_body, B, lane, I0, I1, z0);
}

// BDIM blend of face I of component c: out = V + mu0 f + sum_j mu1_cj
// (f[I+e_j]-f[I-e_j])/2.  CORR = 0: uo = out (predictor); CORR = 1: uo = (u + out)/2
// (corrector).  uo may be u.
template <typename T, int D, int CORR>
__device__ __forceinline__ void bdim_face(const Grid3& g, const Vec3<T>& f, const Vec3<T>& V, const Vec3<T>& mu0,
                                          const Vec9<T>& mu1, const Vec3<T>& u, int has_body, const StdBox& B,
                                          int c, const int I[3], int idx, const Vec3<T>& uo) {
  T acc;
  bool fast = true;
  for (int a = 0; a < D; ++a) fast = fast && I[a] >= 2 && I[a] <= g.n[a] - 1;
  if (has_body && std_point<D>(B, g, I, 0)) {
    acc = L_std<T>(g, B, c, I[c]) * f.c[c][idx];  // V = 0, mu0 = L, mu1 = 0 outside the box
  } else if (has_body && fast) {
    acc = V.c[c][idx] + mu0.c[c][idx] * f.c[c][idx];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = g.s[j];
      acc = acc + mu1.c[c * D + j][idx] * (T(0.5) * (f.c[c][idx + sj] - f.c[c][idx - sj]));
    }
  } else if (has_body) {
    acc = V.c[c][idx] + mu0.c[c][idx] * f.c[c][idx];
    for (int j = 0; j < D; ++j) {
      int Jp[3] = {I[0], I[1], I[2]}, Jm[3] = {I[0], I[1], I[2]};
      const int xp = I[j] + 1, xm = I[j] - 1;
      bool ok = true;
      if (g.per[j]) {
        Jp[j] = wrapc(xp, j, g);
        Jm[j] = wrapc(xm, j, g);
      } else {
        ok = xp <= g.n[j] + 1 && xm >= 0;
        Jp[j] = xp;
        Jm[j] = xm;
      }
      T grad = T(0);
      if (ok)
        grad = T(0.5) * (f.c[c][lin3<T, D>(g, Jp[0], Jp[1], Jp[2])] - f.c[c][lin3<T, D>(g, Jm[0], Jm[1], Jm[2])]);
      acc = acc + mu1.c[c * D + j][idx] * grad;
    }
  } else {
    acc = f.c[c][idx];  // mu0 = 1, mu1 = 0, V = 0 (boundary faces are reset by the BCs)
  }
  if (CORR) uo.c[c][idx] = T(0.5) * (u.c[c][idx] + acc);
  else uo.c[c][idx] = acc;
}

template <typename T, int D, int CORR>
__global__ void __launch_bounds__(kBlock) k_bdim(Grid3 g, Vec3<T> f, Vec3<T> V, Vec3<T> mu0,
                                                 Vec9<T> mu1, Vec3<T> u, int has_body, StdBox B) {
  const int c = blockIdx.y;
  const int P0 = g.n[0] + 2, P1 = g.n[1] + 2, P2 = (D == 3) ? g.n[2] + 2 : 1;
  const int total = P0 * P1 * P2;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I0 = lin % P0, t = lin / P0, I1 = t % P1, I2 = t / P1;
    const int I[3] = {I0, I1, I2};
    bdim_face<T, D, CORR>(g, f, V, mu0, mu1, u, has_body, B, c, I, lin3<T, D>(g, I0, I1, I2), u);
  }
}

// The blend of the faces of the body box [lo, lo + n) (padded indices, 3-D) after a
// fused flux launch (k_flux_reuse with FUSE = 1 + CORR): reads f~, writes uo.
template <typename T, int CORR>
__global__ void __launch_bounds__(kBlock) k_bdim_box(Grid3 g, Vec3<T> f, Vec3<T> V, Vec3<T> mu0, Vec9<T> mu1,
                                                     Vec3<T> u, Vec3<T> uo, StdBox B, int3 lo, int3 n) {
  const int c = blockIdx.y;
  const int64_t total = (int64_t)n.x * n.y * n.z;
  for (int64_t lin = (int64_t)blockIdx.x * kBlock + threadIdx.x; lin < total; lin += (int64_t)gridDim.x * kBlock) {
    const int I[3] = {lo.x + (int)(lin % n.x), lo.y + (int)((lin / n.x) % n.y), lo.z + (int)(lin / ((int64_t)n.x * n.y))};
    bdim_face<T, 3, CORR>(g, f, V, mu0, mu1, u, 1, B, c, I, lin3<T, 3>(g, I[0], I[1], I[2]), uo);
  }
}

// ---------------------------------------------------------------------------
// boundary conditions (closed form of the axis-by-axis rule) and convective exit
// ---------------------------------------------------------------------------
struct Plane {
  int comp, axis, idx;
};
struct Planes {
  Plane p[27];
  int count;
};

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_bc(Grid3 g, Vec3<T> u, Planes pl, double U0, double U1,
                                               double U2, const T* ebuf, const double* scal,
                                               int use_exit) {
  const Plane P = pl.p[blockIdx.y];
  const int c = P.comp, ax = P.axis;
  // the two other axes of the plane
  const int o0 = (ax == 0) ? 1 : 0, o1 = (ax == 2) ? 1 : 2;
  const int m0 = g.n[o0] + 2, m1 = (D == 3) ? g.n[o1] + 2 : 1;
  const int total = m0 * m1;
  const double Uc = (c == 0) ? U0 : (c == 1 ? U1 : U2);
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3] = {0, 0, 0};
    I[ax] = P.idx;
    I[o0] = lin % m0;
    if (D == 3) I[o1] = lin / m0;
    const int idx = lin3<T, D>(g, I[0], I[1], I[2]);
    // source index: ghosts map to the nearest interior (or across the period)
    int S[3] = {I[0], I[1], I[2]};
    for (int a = 0; a < D; ++a) {
      const int N = g.n[a];
      if (I[a] == 0) S[a] = g.per[a] ? N : 1;
      else if (I[a] == N + 1) S[a] = g.per[a] ? 1 : N;
    }
    T val;
    const int Nc = g.n[c];
    if (!g.per[c] && (I[c] <= 1 || I[c] == Nc + 1)) {
      if (use_exit && c == 0 && I[0] == Nc + 1) {
        const int e = S[1] + ((D == 3) ? S[2] * (g.n[1] + 2) : 0);
        val = T(double(ebuf[e]) + scal[kScalExitShift]);
      } else {
        val = T(Uc);
      }
    } else {
      val = u.c[c][lin3<T, D>(g, S[0], S[1], S[2])];
    }
    u.c[c][idx] = val;
  }
}

// exit value e = u0_x[N+1] - dt U (u0_x[N+1] - u0_x[N]) on the interior of the +x plane.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_exit_raw(Grid3 g, const T* u0x, T* ebuf, T dtU, double* part) {
  const int m0 = g.n[1], m1 = (D == 3) ? g.n[2] : 1;
  const int total = m0 * m1;
  const int N = g.n[0];
  double s = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int j = lin % m0 + 1, k = (D == 3) ? lin / m0 + 1 : 0;
    const int base = j * g.s[1] + ((D == 3) ? k * g.s[2] : 0);
    const T ue = u0x[base + N + 1], ub = u0x[base + N];
    const T e = ue - dtU * (ue - ub);
    ebuf[j + ((D == 3) ? k * (g.n[1] + 2) : 0)] = e;
    s += double(e);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// shift = (inlet flux - exit flux)/count  (single block)
__global__ void __launch_bounds__(kBlock) k_exit_shift(const double* part, int nparts, double inlet,
                                                       double count, double* scal) {
  const double s = total_of(part, nparts);
  if (threadIdx.x == 0) scal[kScalExitShift] = (inlet - s) / count;
}

// ---------------------------------------------------------------------------
// projection: divergence + initial residual, multigrid passes, velocity update
// ---------------------------------------------------------------------------
template <int D>
struct Cell {
  int I[3];
  int idx;
};

template <int D>
__device__ __forceinline__ void cell_of(const Grid3& g, int lin, int I[3], int& idx) {
  I[0] = lin % g.n[0] + 1;
  const int t = lin / g.n[0];
  I[1] = t % g.n[1] + 1;
  I[2] = (D == 3) ? t / g.n[1] + 1 : 0;
  idx = I[0] + I[1] * g.s[1] + I[2] * g.s[2];
}

// +/- neighbour offsets of an interior cell (periodic wrap, else ghost)
template <int D>
__device__ __forceinline__ void nbr_offsets(const Grid3& g, const int I[3], int op[3], int om[3]) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    op[a] = (g.per[a] && I[a] == g.n[a]) ? -(g.n[a] - 1) * g.s[a] : g.s[a];
    om[a] = (g.per[a] && I[a] == 1) ? (g.n[a] - 1) * g.s[a] : -g.s[a];
  }
}

// The kernels that hand a residual to a PCG sweep (div_res, restrict, prolong,
// mean0) also emit per-block partials of sum(r) and of the active-cell count
// over active cells: the sweep removes the residual's mean first.
__device__ __forceinline__ void put_mean_partials(double sr, double cnt, double* red) {
  sr = block_sum(sr);
  cnt = block_sum(cnt);
  if (threadIdx.x == 0) {
    red[(size_t)kSlotSumR * kMaxBlocks + blockIdx.x] = sr;
    red[(size_t)kSlotCnt * kMaxBlocks + blockIdx.x] = cnt;
  }
}

// r = z - A x0 on active cells (0 on solid cells), z = rhs or div u, x0 = p wdt (if p) else x.
// Writes x (if p), r; partials: max|r|, sum r, active count; resets the level's PCG flag.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_div_res(Grid3 g, Vec3<T> u, const T* rhs, const T* p,
                                                    T wdt, Vec3<T> L, const T* iD, T* x, T* r,
                                                    double* part_max, double* red, int* flag, StdBox B) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double mx = 0.0, sr = 0.0, cnt = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  const StdDiag<T, D> SD(B);
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, lin, I, idx);
    nbr_offsets<D>(g, I, op, om);
    // every load is issued up front (the coefficients only near the body), so one
    // memory round trip serves the cell
    const bool sc = std_point<D>(B, g, I, 1);
    T di, Lp[3], Lc[3];
    if (sc) {
      di = SD.at(g, I[0], I[1], I[2]);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        Lp[a] = L_std<T>(g, B, a, I[a] + 1);
        Lc[a] = L_std<T>(g, B, a, I[a]);
      }
    } else {
      di = iD[idx];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        Lp[a] = L.c[a][idx + op[a]];
        Lc[a] = L.c[a][idx];
      }
    }
    const T* xs = p ? p : x;
    const T sx = p ? wdt : T(1);
    const T xc = xs[idx] * sx;
    T xp[3], xm[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      xp[a] = xs[idx + op[a]] * sx;
      xm[a] = xs[idx + om[a]] * sx;
    }
    T z;
    if (rhs) {
      z = rhs[idx];
    } else {
      z = T(0);
      for (int a = 0; a < D; ++a) z = z + (u.c[a][idx + op[a]] - u.c[a][idx]);
    }
    T rr = T(0);
    if (di != T(0)) {
      T Ax = T(0);
      for (int a = 0; a < D; ++a) Ax = Ax + Lp[a] * (xp[a] - xc) - Lc[a] * (xc - xm[a]);
      rr = z - Ax;
    }
    if (p) x[idx] = xc;
    r[idx] = rr;
    mx = fmax(mx, fabs(double(rr)));
    if (di != T(0)) {
      sr += double(rr);
      cnt += 1.0;
    }
  }
  mx = block_max(mx);
  if (threadIdx.x == 0) part_max[blockIdx.x] = mx;
  put_mean_partials(sr, cnt, red);
}

// mean partials of the current residual (used when the grid has a single level)
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_mean0(Grid3 g, const T* iD, const T* r, double* red, int* flag) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double sr = 0.0, cnt = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    if (iD[idx] != T(0)) {
      sr += double(r[idx]);
      cnt += 1.0;
    }
  }
  put_mean_partials(sr, cnt, red);
}

// restriction: r_c = sum of the 2^D children (0 on solid coarse cells), x_c = 0; rho partial.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_restrict(Grid3 f, Grid3 c, const T* rf, const T* iDc, T* rc,
                                                     T* xc, double* red, int* flag) {
  const int total = c.n[0] * c.n[1] * ((D == 3) ? c.n[2] : 1);
  double sr = 0.0, cnt = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int J[3], cidx;
    cell_of<D>(c, lin, J, cidx);
    int base = (2 * J[0] - 1) + (2 * J[1] - 1) * f.s[1] + ((D == 3) ? (2 * J[2] - 1) * f.s[2] : 0);
    T s = rf[base] + rf[base + 1] + rf[base + f.s[1]] + rf[base + 1 + f.s[1]];
    if (D == 3) {
      const int b2 = base + f.s[2];
      s = s + (rf[b2] + rf[b2 + 1] + rf[b2 + f.s[1]] + rf[b2 + 1 + f.s[1]]);
    }
    const T di = iDc[cidx];
    const T rr = (di != T(0)) ? s : T(0);
    rc[cidx] = rr;
    xc[cidx] = T(0);
    if (di != T(0)) {
      sr += double(rr);
      cnt += 1.0;
    }
  }
  put_mean_partials(sr, cnt, red);
}

// prolongation + correction: e = x_c[parent]; x_f += e; r_f -= A_f e; rho partial.
template <typename T, int D>
__device__ __forceinline__ int parent_idx(const Grid3& c, int I0, int I1, int I2) {
  // fine padded coordinate -> coarse padded coordinate (ghosts map to ghosts)
  return ((I0 + 1) >> 1) + ((I1 + 1) >> 1) * c.s[1] + ((D == 3) ? ((I2 + 1) >> 1) * c.s[2] : 0);
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_prolong(Grid3 f, Grid3 c, const T* xc, Vec3<T> L, const T* iD,
                                                    T* xf, T* rf, double* red, int* flag) {
  const int total = f.n[0] * f.n[1] * ((D == 3) ? f.n[2] : 1);
  double sr = 0.0, cnt = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(f, lin, I, idx);
    const T ec = xc[parent_idx<T, D>(c, I[0], I[1], I[2])];
    xf[idx] = xf[idx] + ec;
    const T di = iD[idx];
    T rr = rf[idx];
    if (di != T(0)) {
      T Ae = T(0);
      for (int a = 0; a < D; ++a) {
        int Jp[3] = {I[0], I[1], I[2]}, Jm[3] = {I[0], I[1], I[2]};
        Jp[a] = wrapc(I[a] + 1, a, f);
        Jm[a] = wrapc(I[a] - 1, a, f);
        const T ep = xc[parent_idx<T, D>(c, Jp[0], Jp[1], Jp[2])];
        const T em = xc[parent_idx<T, D>(c, Jm[0], Jm[1], Jm[2])];
        const int op = (f.per[a] && I[a] == f.n[a]) ? -(f.n[a] - 1) * f.s[a] : f.s[a];
        Ae = Ae + L.c[a][idx + op] * (ep - ec) - L.c[a][idx] * (ec - em);
      }
      rr = rr - Ae;
      rf[idx] = rr;
      sr += double(rr);
      cnt += 1.0;
    }
  }
  put_mean_partials(sr, cnt, red);
}

// Prolongation + correction, tiled z-marching form for large 3-D levels (same tile
// order as the tiled PCG pass A): e = x_c[parent]; x += e; r -= A e; mean partials.
// Like the PCG marches: branch-free loads issued two planes ahead, one marching body
// per coefficient mode.
template <typename T, bool FAST>
__device__ __forceinline__ void prolong_march(const Grid3& f, const Grid3& c, const T* __restrict__ xc,
                                              const Vec3<T>& L, const T* __restrict__ iD, T* __restrict__ xf,
                                              T* __restrict__ rf, const StdBox& B, int i, int j, int z0, int z1,
                                              double& sr, double& cnt) {
  const StdDiag<T, 3> SD(B);
  const int s1 = f.s[1], s2 = f.s[2], cs1 = c.s[1], cs2 = c.s[2];
  const int col = i + j * s1;
  const int pi = (i + 1) >> 1, pj = (j + 1) >> 1;
  const int pxp = (wrapc(i + 1, 0, f) + 1) >> 1, pxm = (wrapc(i - 1, 0, f) + 1) >> 1;
  const int pyp = (wrapc(j + 1, 1, f) + 1) >> 1, pym = (wrapc(j - 1, 1, f) + 1) >> 1;
  const int cc = pi + pj * cs1, cxp = pxp + pj * cs1, cxm = pxm + pj * cs1, cyp = pi + pyp * cs1,
            cym = pi + pym * cs1;
  const int opx = (f.per[0] && i == f.n[0]) ? -(f.n[0] - 1) : 1;
  const int opy = (f.per[1] && j == f.n[1]) ? -(f.n[1] - 1) * s1 : s1;
  const T Lxp0 = L_std<T>(f, B, 0, i + 1), Lxc0 = L_std<T>(f, B, 0, i);
  const T Lyp0 = L_std<T>(f, B, 1, j + 1), Lyc0 = L_std<T>(f, B, 1, j);
  struct Raw {
    T x, r, d, e, exp, exm, eyp, eym, ezp, ezm, lxp, lxc, lyp, lyc, lzp, lzc;
  };
  auto load = [&](int zz) -> Raw {
    const int z = min(zz, f.n[2]);  // planes past the tile are clamped (not used)
    const int id = col + z * s2;
    const int zp = wrapc(z + 1, 2, f), zm = wrapc(z - 1, 2, f);
    const int pz = ((z + 1) >> 1) * cs2, pzp = ((zp + 1) >> 1) * cs2, pzm = ((zm + 1) >> 1) * cs2;
    Raw v;
    v.x = xf[id];
    v.r = rf[id];
    v.e = xc[cc + pz];
    v.exp = xc[cxp + pz];
    v.exm = xc[cxm + pz];
    v.eyp = xc[cyp + pz];
    v.eym = xc[cym + pz];
    v.ezp = xc[cc + pzp];
    v.ezm = xc[cc + pzm];
    if (FAST) {
      v.d = SD.at(f, i, j, z);
      v.lxp = Lxp0;
      v.lxc = Lxc0;
      v.lyp = Lyp0;
      v.lyc = Lyc0;
      v.lzp = L_std<T>(f, B, 2, zp);
      v.lzc = L_std<T>(f, B, 2, z);
    } else {
      v.d = iD[id];
      v.lxp = L.c[0][id + opx];
      v.lxc = L.c[0][id];
      v.lyp = L.c[1][id + opy];
      v.lyc = L.c[1][id];
      v.lzp = L.c[2][col + zp * s2];
      v.lzc = L.c[2][id];
    }
    return v;
  };
  auto plane = [&](int z, const Raw& v, Raw& nxt) {
    nxt = load(z + 2);
    const int id = col + z * s2;
    xf[id] = v.x + v.e;
    if (v.d != T(0)) {
      T Ae = T(0);
      Ae = Ae + v.lxp * (v.exp - v.e) - v.lxc * (v.e - v.exm);
      Ae = Ae + v.lyp * (v.eyp - v.e) - v.lyc * (v.e - v.eym);
      Ae = Ae + v.lzp * (v.ezp - v.e) - v.lzc * (v.e - v.ezm);
      const T rr = v.r - Ae;
      rf[id] = rr;
      sr += double(rr);
      cnt += 1.0;
    }
  };
  Raw A = load(z0), Bn = load(z0 + 1), C;
  for (int z = z0; z < z1; z += 3) {
    plane(z, A, C);
    if (z + 1 >= z1) break;
    plane(z + 1, Bn, A);
    if (z + 2 >= z1) break;
    plane(z + 2, C, Bn);
  }
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_prolong_tile(Grid3 f, Grid3 c, const T* xc, Vec3<T> L, const T* iD,
                                                      T* xf, T* rf, double* red, int* flag, int tiles_x,
                                                      int tiles_y, int ntiles, int tz, StdBox B) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  const int b = blockIdx.x;
  const int full = (ntiles / 8) * 8;
  const int tile = (b < full) ? (b % 8) * (ntiles / 8) + b / 8 : b;
  const int txi = tile % tiles_x, rem = tile / tiles_x, tyi = rem % tiles_y, tzi = rem / tiles_y;
  const int x0 = 1 + txi * kTX, y0 = 1 + tyi * kTY, z0 = 1 + tzi * tz;
  const int z1 = min(z0 + tz, f.n[2] + 1);
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int i = x0 + tx, j = y0 + ty;
  const bool own = i <= f.n[0] && j <= f.n[1];
  const int ta[3] = {x0 - 2, y0 - 2, z0 - 2}, tb[3] = {x0 + kTX + 1, y0 + kTY + 1, z1 + 1};
  const bool fast = std_miss<3>(B, f, ta, tb);  // L and iD in closed form
  double sr = 0.0, cnt = 0.0;
  if (own) {
    if (fast)
      prolong_march<T, true>(f, c, xc, L, iD, xf, rf, B, i, j, z0, z1, sr, cnt);
    else
      prolong_march<T, false>(f, c, xc, L, iD, xf, rf, B, i, j, z0, z1, sr, cnt);
  }
  sr = block_sum<kTileThreads>(sr);
  cnt = block_sum<kTileThreads>(cnt);
  if (threadIdx.x == 0) {
    red[(size_t)kSlotSumR * kMaxBlocks + blockIdx.x] = sr;
    red[(size_t)kSlotCnt * kMaxBlocks + blockIdx.x] = cnt;
  }
}

// mean of the residual over the active cells, from the producer's partials
template <int NT = kBlock>
__device__ __forceinline__ double residual_mean(const double* red, int nparts) {
  const double cnt = total_of<NT>(red + (size_t)kSlotCnt * kMaxBlocks, nparts);
  const double sr = total_of<NT>(red + (size_t)kSlotSumR * kMaxBlocks, nparts);
  return cnt > 0.0 ? sr / cnt : 0.0;
}

// Scalars of PCG pass A at sweep k: beta (k > 0) or the residual mean (k = 0).
// Returns false (and sets the stop flag) when rho_k == 0 for k > 0.
template <typename T, int NT>
__device__ __forceinline__ bool pcg_a_scalars(const double* red, int k, const RedN& rn, int* flag, T& beta,
                                              T& mean) {
  beta = T(0);
  mean = T(0);
  if (k > 0) {
    const double rho = total_of<NT>(red + (size_t)(kSlotRho0 + k) * kMaxBlocks, rn.rho);
    if (rho == 0.0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
      return false;
    }
    beta = T(rho / total_of<NT>(red + (size_t)(kSlotRho0 + k - 1) * kMaxBlocks, rn.rho_prev));
  } else {
    mean = T(residual_mean<NT>(red, rn.mean));
  }
  return true;
}

// PCG pass A (sweep k), generic grid-stride form.  k = 0: e = iD (r - m) with m the
// residual mean over active cells, rho_0 partial = sum (r - m) e.  k > 0:
// e_new = iD r + beta e_old, beta = rho_k/rho_{k-1} (stops if rho_k == 0).  Then
// q = A e_new (0 on solid cells) and the sigma partial = sum e_new q.
// FINE = 1 only makes the fine-level launches a separate kernel symbol in traces.
template <typename T, int D, int FINE>
__global__ void __launch_bounds__(kBlock) k_pcg_a(Grid3 g, Vec3<T> L, const T* iD, const T* r, const T* eo,
                                                  T* en, T* q, double* red, int k, RedN rn,
                                                  double* part_sig, int* flag) {
  if (*flag) return;
  T beta, mean;
  if (!pcg_a_scalars<T, kBlock>(red, k, rn, flag, beta, mean)) return;
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double sig = 0.0, rho0 = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, lin, I, idx);
    nbr_offsets<D>(g, I, op, om);
    const T di = iD[idx];
    const T ec = (k > 0) ? di * r[idx] + beta * eo[idx] : di * (r[idx] - mean);
    en[idx] = ec;
    T qq = T(0);
    if (di != T(0)) {
      for (int a = 0; a < D; ++a) {
        const int ip = idx + op[a], im = idx + om[a];
        const T ep = (k > 0) ? iD[ip] * r[ip] + beta * eo[ip] : iD[ip] * (r[ip] - mean);
        const T em = (k > 0) ? iD[im] * r[im] + beta * eo[im] : iD[im] * (r[im] - mean);
        qq = qq + L.c[a][ip] * (ep - ec) - L.c[a][idx] * (ec - em);
      }
      if (k == 0) rho0 += double(r[idx] - mean) * double(ec);
    }
    q[idx] = qq;
    sig += double(ec) * double(qq);
  }
  sig = block_sum(sig);
  if (threadIdx.x == 0) part_sig[blockIdx.x] = sig;
  if (k == 0) {
    rho0 = block_sum(rho0);
    if (threadIdx.x == 0) red[(size_t)kSlotRho0 * kMaxBlocks + blockIdx.x] = rho0;
  }
}

// ---------------------------------------------------------------------------
// 2.5-D tiles of the large 3-D levels: one block of 64 x 8 threads per
// (64 x 8 x kTZ) column stack, marching in z.  The values of the current plane
// (tile + a one-cell ring) live in a double-buffered LDS plane, the planes z-1 and
// z+1 of the block's own columns in registers; loads for the next planes are
// issued one iteration ahead, so one barrier per plane suffices and the load
// latency overlaps the stencil work.
// ---------------------------------------------------------------------------
struct TileGeo {
  int x0, y0, z0, z1;  // tile origin and end plane (exclusive)
  int tx, ty, i, j;    // own column
  bool inb, own;       // column inside the padded grid / interior
  int col;             // wrapped linear index of the own column (z = 0)
  bool ring;           // this thread also carries one ring cell
  int sx, sy, hx, hy;  // ring cell: LDS position, wrapped grid coordinates
  bool hb;             // ring cell inside the padded grid
  int hcol;
  int opx, opy;        // +x / +y face offsets of the own column (periodic wrap)
  bool fast;           // the stencil misses the body box: closed-form coefficients

  __device__ TileGeo(const Grid3& g, const StdBox& B, int tiles_x, int tiles_y, int ntiles, int tz) {
    // XCD-aware tile order: consecutive hardware blocks round-robin over the 8 XCDs,
    // so give each XCD a contiguous range of tiles (shared halos stay in its L2)
    const int b = blockIdx.x;
    const int full = (ntiles / 8) * 8;
    const int tile = (b < full) ? (b % 8) * (ntiles / 8) + b / 8 : b;
    const int txi = tile % tiles_x, rem = tile / tiles_x, tyi = rem % tiles_y, tzi = rem / tiles_y;
    x0 = 1 + txi * kTX;
    y0 = 1 + tyi * kTY;
    z0 = 1 + tzi * tz;
    z1 = min(z0 + tz, g.n[2] + 1);
    tx = threadIdx.x % kTX;
    ty = threadIdx.x / kTX;
    i = x0 + tx;
    j = y0 + ty;
    const int n0 = g.n[0], n1 = g.n[1];
    inb = i <= n0 + 1 && j <= n1 + 1;
    own = i <= n0 && j <= n1;
    col = wrapc(i, 0, g) + wrapc(j, 1, g) * g.s[1];
    const int t = threadIdx.x;
    ring = t < 2 * (kTX + 2) + 2 * kTY;
    sx = sy = hx = hy = hcol = 0;
    hb = false;
    if (ring) {
      if (t < kTX + 2) {
        sx = t;
        sy = 0;
      } else if (t < 2 * (kTX + 2)) {
        sx = t - (kTX + 2);
        sy = kTY + 1;
      } else if (t < 2 * (kTX + 2) + kTY) {
        sx = 0;
        sy = 1 + t - 2 * (kTX + 2);
      } else {
        sx = kTX + 1;
        sy = 1 + t - 2 * (kTX + 2) - kTY;
      }
      const int rx = x0 - 1 + sx, ry = y0 - 1 + sy;
      hb = rx >= 0 && rx <= n0 + 1 && ry >= 0 && ry <= n1 + 1;
      hx = wrapc(rx, 0, g);
      hy = wrapc(ry, 1, g);
      hcol = hx + hy * g.s[1];
    }
    opx = (g.per[0] && i == n0) ? -(n0 - 1) : 1;
    opy = (g.per[1] && j == n1) ? -(n1 - 1) * g.s[1] : g.s[1];
    const int ta[3] = {x0 - 2, y0 - 2, z0 - 2}, tb[3] = {x0 + kTX + 1, y0 + kTY + 1, z1 + 1};
    fast = std_miss<3>(B, g, ta, tb);
  }
};

// The march loads every plane branch-free from clamped (always valid) addresses
// and selects afterwards, with one marching body per coefficient mode (closed
// form or loaded): loads behind data-dependent branches would each be waited for
// at the branch's join, which serialises the march on memory latency.  Loads run
// two planes ahead of their use.
__device__ __forceinline__ int clamp_plane(const Grid3& g, int z) {
  return wrapc(min(max(z, 0), g.n[2] + 1), 2, g);
}

template <typename T, int STOREQ, bool FAST>
__device__ __forceinline__ void pcg_a_march(const Grid3& g, const Vec3<T>& L, const T* __restrict__ iD,
                                            const T* __restrict__ r, const T* __restrict__ eo, T* __restrict__ en,
                                            T* __restrict__ q, int k, T beta, T mean, const TileGeo& G,
                                            const StdBox& B, T (*sE)[kTY + 2][kTX + 2], double& sig,
                                            double& rho0) {
  const StdDiag<T, 3> SD(B);
  const int s1 = g.s[1], s2 = g.s[2];
  // clamped columns: threads outside the padded grid read a valid column, unused
  const int ci = min(G.i, g.n[0] + 1), cj = min(G.j, g.n[1] + 1);
  const int wi = wrapc(ci, 0, g), wj = wrapc(cj, 1, g);
  const int col = wi + wj * s1;
  const int hcol = G.hb ? G.hcol : col;
  const bool use_ring = G.ring && G.hb;
  auto eps3 = [&](T d, T rv, T ev) -> T { return (k > 0) ? d * rv + beta * ev : d * (rv - mean); };
  // raw loads of one plane; e is formed only when the plane is used, so a load is
  // waited for two iterations after it was issued
  struct Raw {
    T d, r, e, l;
  };
  // planes past the tile's last needed one (z1 for the own column, z1-1 for the
  // ring) re-read that plane, a cache hit, instead of fetching unused data
  auto own = [&](int zz) -> Raw {
    const int zw = clamp_plane(g, min(zz, G.z1)), id = col + zw * s2;
    Raw v;
    v.r = r[id];
    v.e = eo[id];
    v.d = FAST ? SD.at(g, wi, wj, zw) : iD[id];
    v.l = FAST ? L_std<T>(g, B, 2, zw) : L.c[2][id];
    return v;
  };
  auto ring = [&](int zz) -> Raw {
    const int zw = clamp_plane(g, min(zz, G.z1 - 1)), id = hcol + zw * s2;
    Raw v;
    v.r = r[id];
    v.e = eo[id];
    v.d = FAST ? SD.at(g, G.hx, G.hy, zw) : iD[id];
    v.l = T(0);
    return v;
  };
  const T Lxp0 = L_std<T>(g, B, 0, G.i + 1), Lxc0 = L_std<T>(g, B, 0, G.i);
  const T Lyp0 = L_std<T>(g, B, 1, G.j + 1), Lyc0 = L_std<T>(g, B, 1, G.j);
  const Raw am = own(G.z0 - 1), a0 = own(G.z0);
  T em = eps3(am.d, am.r, am.e), ec = eps3(a0.d, a0.r, a0.e), dc = a0.d, rc = a0.r, L2c = a0.l;
  // one plane: consumes own plane z+1 (ap) and ring plane z (hr), issues the loads
  // of own plane z+1+kPF and ring plane z+kPF (used kPF planes later)
  auto plane = [&](int z, const Raw& ap, const Raw& hr, Raw& a_new, Raw& h_new) {
    a_new = own(z + 1 + kPF);
    h_new = ring(z + kPF);
    const T ep = eps3(ap.d, ap.r, ap.e), L2p = ap.l;
    T(*P)[kTX + 2] = sE[z & 1];
    P[G.ty + 1][G.tx + 1] = ec;
    if (G.ring) P[G.sy][G.sx] = use_ring ? eps3(hr.d, hr.r, hr.e) : T(0);
    __syncthreads();
    if (G.own) {
      const int id = col + z * s2;
      T qq = T(0);
      if (dc != T(0)) {
        const T xm = P[G.ty + 1][G.tx], xp = P[G.ty + 1][G.tx + 2];
        const T ym = P[G.ty][G.tx + 1], yp = P[G.ty + 2][G.tx + 1];
        const T Lxp = FAST ? Lxp0 : L.c[0][id + G.opx], Lxc = FAST ? Lxc0 : L.c[0][id];
        const T Lyp = FAST ? Lyp0 : L.c[1][id + G.opy], Lyc = FAST ? Lyc0 : L.c[1][id];
        qq = qq + Lxp * (xp - ec) - Lxc * (ec - xm);
        qq = qq + Lyp * (yp - ec) - Lyc * (ec - ym);
        qq = qq + L2p * (ep - ec) - L2c * (ec - em);
        if (k == 0) rho0 += double(rc - mean) * double(ec);
      }
      st_stream(en + id, ec);
      if (STOREQ) q[id] = qq;
      sig += double(ec) * double(qq);
    }
    // the other LDS buffer is written next: no second barrier
    em = ec;
    ec = ep;
    dc = ap.d;
    rc = ap.r;
    L2c = L2p;
  };
  // kPF + 1 planes per trip over kPF + 1 register slots indexed by constants, so
  // the slots are renamed rather than copied (a copy of a register whose load is
  // in flight would wait for it): own plane z0+1+m lives in S[m % NS], ring
  // plane z0+m in H[m % NS]
  constexpr int NS = kPF + 1;
  Raw S[NS], H[NS];
#pragma unroll
  for (int m = 0; m < kPF; ++m) {
    S[m] = own(G.z0 + 1 + m);
    H[m] = ring(G.z0 + m);
  }
  for (int z = G.z0; z < G.z1; z += NS) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      if (z + u >= G.z1) break;
      plane(z + u, S[u], H[u], S[(u + kPF) % NS], H[(u + kPF) % NS]);
    }
  }
}

// PCG pass A, tiled form (see k_pcg_a for the arithmetic).  With STOREQ = 0,
// q = A e is only reduced into sigma, not stored: the tiled pass B recomputes it.
template <typename T, int FINE, int STOREQ = 1>
__global__ void __launch_bounds__(kTileThreads) k_pcg_a_tile(Grid3 g, Vec3<T> L, const T* iD, const T* r,
                                                             const T* eo, T* en, T* q, double* red, int k,
                                                             RedN rn, double* part_sig, int* flag, int tiles_x,
                                                             int tiles_y, int ntiles, int tz, StdBox B) {
  if (*flag) return;
  T beta, mean;
  if (!pcg_a_scalars<T, kTileThreads>(red, k, rn, flag, beta, mean)) return;
  __shared__ T sE[2][kTY + 2][kTX + 2];
  const TileGeo G(g, B, tiles_x, tiles_y, ntiles, tz);
  double sig = 0.0, rho0 = 0.0;
  if (G.fast)
    pcg_a_march<T, STOREQ, true>(g, L, iD, r, eo, en, q, k, beta, mean, G, B, sE, sig, rho0);
  else
    pcg_a_march<T, STOREQ, false>(g, L, iD, r, eo, en, q, k, beta, mean, G, B, sE, sig, rho0);
  sig = block_sum<kTileThreads>(sig);
  if (threadIdx.x == 0) part_sig[blockIdx.x] = sig;
  if (k == 0) {
    rho0 = block_sum<kTileThreads>(rho0);
    if (threadIdx.x == 0) red[(size_t)kSlotRho0 * kMaxBlocks + blockIdx.x] = rho0;
  }
}

// PCG pass B march (see k_pcg_b_tile)
template <typename T, bool FAST>
__device__ __forceinline__ void pcg_b_march(const Grid3& g, const Vec3<T>& L, const T* __restrict__ iD,
                                            const T* __restrict__ e, T* __restrict__ x, T* __restrict__ r, T alpha,
                                            T mean, bool skip, const TileGeo& G, const StdBox& B,
                                            T (*sE)[kTY + 2][kTX + 2], double& rho, double& mx) {
  const StdDiag<T, 3> SD(B);
  const int s1 = g.s[1], s2 = g.s[2];
  const int ci = min(G.i, g.n[0] + 1), cj = min(G.j, g.n[1] + 1);
  const int wi = wrapc(ci, 0, g), wj = wrapc(cj, 1, g);
  const int col = wi + wj * s1;
  const int hcol = G.hb ? G.hcol : col;
  const bool use_ring = G.ring && G.hb;
  // own column: e and L_z, x, r, iD of a plane (raw: used two iterations later)
  struct Raw {
    T e, l, x, r, d;
  };
  auto own = [&](int zz) -> Raw {
    const int zw = clamp_plane(g, min(zz, G.z1)), id = col + zw * s2;  // see pcg_a_march
    Raw v;
    v.e = e[id];
    v.l = FAST ? L_std<T>(g, B, 2, zw) : L.c[2][id];
    v.x = ld_stream(x + id);
    v.r = ld_stream(r + id);
    v.d = FAST ? SD.at(g, wi, wj, zw) : iD[id];
    return v;
  };
  auto ring = [&](int zz) -> T { return e[hcol + clamp_plane(g, min(zz, G.z1 - 1)) * s2]; };
  const T Lxp0 = L_std<T>(g, B, 0, G.i + 1), Lxc0 = L_std<T>(g, B, 0, G.i);
  const T Lyp0 = L_std<T>(g, B, 1, G.j + 1), Lyc0 = L_std<T>(g, B, 1, G.j);
  T em = own(G.z0 - 1).e;
  // one plane: consumes own planes z (cur) and z+1 (nxt) and ring plane z (hr),
  // issues the loads of own plane z+kPF and ring plane z+kPF
  auto plane = [&](int z, const Raw& cur, const Raw& nxt, const T& hr, Raw& a_new, T& h_new) {
    a_new = own(z + kPF);
    h_new = ring(z + kPF);
    const T ec = cur.e, ep = nxt.e, L2c = cur.l, L2p = nxt.l, dc = cur.d;
    T(*P)[kTX + 2] = sE[z & 1];
    P[G.ty + 1][G.tx + 1] = ec;
    if (G.ring) P[G.sy][G.sx] = use_ring ? hr : T(0);
    __syncthreads();
    if (G.own) {
      const int id = col + z * s2;
      T rr = cur.r;
      if (mean != T(0) && dc != T(0)) rr = rr - mean;
      if (!skip) {
        T qq = T(0);
        if (dc != T(0)) {
          const T xm = P[G.ty + 1][G.tx], xp = P[G.ty + 1][G.tx + 2];
          const T ym = P[G.ty][G.tx + 1], yp = P[G.ty + 2][G.tx + 1];
          const T Lxp = FAST ? Lxp0 : L.c[0][id + G.opx], Lxc = FAST ? Lxc0 : L.c[0][id];
          const T Lyp = FAST ? Lyp0 : L.c[1][id + G.opy], Lyc = FAST ? Lyc0 : L.c[1][id];
          qq = qq + Lxp * (xp - ec) - Lxc * (ec - xm);
          qq = qq + Lyp * (yp - ec) - Lyc * (ec - ym);
          qq = qq + L2p * (ep - ec) - L2c * (ec - em);
        }
        st_stream(x + id, cur.x + alpha * ec);
        rr = rr - alpha * qq;
      }
      if (!skip || mean != T(0)) st_stream(r + id, rr);
      rho += double(rr) * (double(dc) * double(rr));
      mx = fmax(mx, fabs(double(rr)));
    }
    em = ec;
  };
  // slots as in pcg_a_march: own plane z0+m in S[m % NS], ring plane z0+m in H[m % NS]
  constexpr int NS = kPF + 1;
  Raw S[NS];
  T H[NS];
#pragma unroll
  for (int m = 0; m < kPF; ++m) {
    S[m] = own(G.z0 + m);
    H[m] = ring(G.z0 + m);
  }
  for (int z = G.z0; z < G.z1; z += NS) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      if (z + u >= G.z1) break;
      plane(z + u, S[u], S[(u + 1) % NS], H[u], S[(u + kPF) % NS], H[(u + kPF) % NS]);
    }
  }
}

// PCG pass B (sweep k), tiled form paired with pass A (STOREQ = 0): q = A e is
// recomputed from e instead of being stored and re-read; then x += alpha e,
// r -= alpha q on the interior, with the same scalars, stopping rule, mean removal
// (sweep 0) and partials (rho_{k+1}, max|r|) as the flat pass B.
template <typename T, int FINE>
__global__ void __launch_bounds__(kTileThreads) k_pcg_b_tile(Grid3 g, Vec3<T> L, const T* iD, const T* e, T* x,
                                                             T* r, double* red, int k, RedN rn, double* part_rho_next,
                                                             double* part_max, int want_rho, int want_max, int* flag,
                                                             int tiles_x, int tiles_y, int ntiles, int tz, StdBox B) {
  bool skip = (*flag) != 0;
  T alpha = T(0);
  const T mean = (k == 0) ? T(residual_mean<kTileThreads>(red, rn.mean)) : T(0);
  if (!skip) {
    const double sig = total_of<kTileThreads>(red + (size_t)(kSlotSig0 + k) * kMaxBlocks, rn.sig);
    if (fabs(sig) < 1e-300) {
      skip = true;
      if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
    } else {
      alpha = T(total_of<kTileThreads>(red + (size_t)(kSlotRho0 + k) * kMaxBlocks, rn.rho) / sig);
    }
  }
  if (skip && !want_max && mean == T(0)) return;  // grid-uniform
  __shared__ T sE[2][kTY + 2][kTX + 2];
  const TileGeo G(g, B, tiles_x, tiles_y, ntiles, tz);
  double rho = 0.0, mx = 0.0;
  if (G.fast)
    pcg_b_march<T, true>(g, L, iD, e, x, r, alpha, mean, skip, G, B, sE, rho, mx);
  else
    pcg_b_march<T, false>(g, L, iD, e, x, r, alpha, mean, skip, G, B, sE, rho, mx);
  if (want_rho && !skip) {
    rho = block_sum<kTileThreads>(rho);
    if (threadIdx.x == 0) part_rho_next[blockIdx.x] = rho;
  }
  if (want_max) {
    mx = block_max<kTileThreads>(mx);
    if (threadIdx.x == 0) part_max[blockIdx.x] = mx;
  }
}

// PCG pass B (sweep k), flat and vectorised over the whole padded array (ghost and
// padding cells have iD = e = q = 0, so they are left unchanged):
// alpha = rho_k/sigma_k; x += alpha e; r -= alpha q; partials rho_{k+1}
// (want_rho) and max|r| (want_max).  Sweep 0 also removes the residual mean from
// r on active cells.  Stops if |sigma| < 1e-300.  Vectors whose cells all lie
// outside the body box (with a one-cell margin) take iD in closed form.
template <typename T, int D, int FINE>
__global__ void __launch_bounds__(kBlock) k_pcg_b(int64_t nvec, const T* iD, const T* e, const T* q, T* x,
                                                  T* r, double* red, int k, RedN rn, double* part_rho_next,
                                                  double* part_max, int want_rho, int want_max, int* flag,
                                                  Grid3 g, StdBox B) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  bool skip = (*flag) != 0;
  T alpha = T(0);
  const T mean = (k == 0) ? T(residual_mean(red, rn.mean)) : T(0);
  if (!skip) {
    const double sig = total_of(red + (size_t)(kSlotSig0 + k) * kMaxBlocks, rn.sig);
    if (fabs(sig) < 1e-300) {
      skip = true;
      if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
    } else {
      alpha = T(total_of(red + (size_t)(kSlotRho0 + k) * kMaxBlocks, rn.rho) / sig);
    }
  }
  if (skip && !want_max && mean == T(0)) return;
  double rho = 0.0, mx = 0.0;
  const V* iDv = reinterpret_cast<const V*>(iD);
  const V* ev = reinterpret_cast<const V*>(e);
  const V* qv = reinterpret_cast<const V*>(q);
  V* xv = reinterpret_cast<V*>(x);
  V* rv = reinterpret_cast<V*>(r);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int px = g.s[1], py = g.n[1] + 2;
  const StdDiag<T, D> SD(B);
  // iD of the W cells of vector v in closed form; false if any of them is near the box
  auto std_vec = [&](int64_t v, V& out) -> bool {
    T* o = reinterpret_cast<T*>(&out);
    const int e0 = (int)(v * W) - kFrontPad;  // field index of lane 0 (< 2^31 by the plan)
    int cx = -1, cy = 0, cz = 0;
    if (e0 >= 0) {
      const int row = e0 / px;
      cx = e0 - row * px;
      cy = row % py;
      cz = row / py;
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      int I[3] = {cx + w, cy, cz};
      if (e0 + w < 0) {
        o[w] = T(0);
        continue;
      }
      if (I[0] >= px) {  // the vector crosses into the next row
        I[0] -= px;
        if (++I[1] == py) {
          I[1] = 0;
          ++I[2];
        }
      }
      if (!std_point<D>(B, g, I, 1)) return false;
      o[w] = SD.at(g, I[0], I[1], I[2]);
    }
    return true;
  };
  // two vectors per thread and trip, both coalesced, so twice the loads are in flight
  for (int64_t v0 = blockIdx.x * (int64_t)kBlock + threadIdx.x; v0 < nvec; v0 += 2 * stride) {
    const int64_t vv[2] = {v0, v0 + stride};
    const bool has[2] = {true, v0 + stride < nvec};
    V dv[2], rr[2], ee[2], qq[2], xx[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!has[h]) continue;
      if (!std_vec(vv[h], dv[h])) dv[h] = iDv[vv[h]];
      rr[h] = rv[vv[h]];
      if (!skip) {
        ee[h] = ev[vv[h]];
        qq[h] = qv[vv[h]];
        xx[h] = xv[vv[h]];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!has[h]) continue;
      T* rs = reinterpret_cast<T*>(&rr[h]);
      const T* ds = reinterpret_cast<const T*>(&dv[h]);
      if (mean != T(0)) {
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (ds[w] != T(0)) rs[w] = rs[w] - mean;
      }
      if (!skip) {
        const T* es = reinterpret_cast<const T*>(&ee[h]);
        const T* qs = reinterpret_cast<const T*>(&qq[h]);
        T* xs = reinterpret_cast<T*>(&xx[h]);
#pragma unroll
        for (int w = 0; w < W; ++w) {
          xs[w] = xs[w] + alpha * es[w];
          rs[w] = rs[w] - alpha * qs[w];
        }
        xv[vv[h]] = xx[h];
      }
      if (!skip || mean != T(0)) rv[vv[h]] = rr[h];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        rho += double(rs[w]) * (double(ds[w]) * double(rs[w]));
        mx = fmax(mx, fabs(double(rs[w])));
      }
    }
  }
  if (want_rho && !skip) {
    rho = block_sum(rho);
    if (threadIdx.x == 0) part_rho_next[blockIdx.x] = rho;
  }
  if (want_max) {
    mx = block_max(mx);
    if (threadIdx.x == 0) part_max[blockIdx.x] = mx;
  }
}

// ---------------------------------------------------------------------------
// The smallest multigrid levels in one workgroup.  Below a few thousand cells a
// level's passes are dominated by launch and reduction overhead, so from level
// Lb down the whole remaining cycle runs in a single block of kBottom threads:
// restriction down to the coarsest level, PCG there, then prolongation +
// correction and PCG on the way up -- the same arithmetic as the per-level
// kernels (the reductions are block-wide instead of per-block partials, so sums
// differ only in rounding order).  During a level's PCG each thread keeps its
// cells' x, r, q, iD and face coefficients in registers and the search
// direction lives in LDS (a compact copy of the padded level, ghosts zero), so
// the sweeps touch no global memory.
// ---------------------------------------------------------------------------
constexpr int kBottom = 1024;
constexpr int kBottomCPT = 4;                          // cells per thread
constexpr int kBottomCells = kBottom * kBottomCPT;     // a level this small or smaller joins the bottom solve
constexpr int kBottomLdsBytes = 49152;                 // LDS for the search direction of one level
template <typename T>
constexpr int bottom_lds_elems() { return kBottomLdsBytes / (int)sizeof(T); }

template <typename T>
struct LevelRef {
  Grid3 g;
  T *x, *r, *e, *q;
  const T* iD;
  Vec3<T> L;
};
constexpr int kBottomMax = 8;  // levels a bottom solve may hold (passed by value)
template <typename T>
struct BottomLevels {
  int n, pcg_iters;          // levels lv[0] (the first bottom level) .. lv[n-1] (coarsest)
  LevelRef<T> lv[kBottomMax];
};

// two block sums for the price of one set of barriers
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sh2[2][NT / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh2[0][w] = a;
    sh2[1][w] = b;
  }
  __syncthreads();
  double ra = sh2[0][0], rb = sh2[1][0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    ra += sh2[0][i];
    rb += sh2[1][i];
  }
  __syncthreads();
  a = ra;
  b = rb;
}

// PCG(K) on one level with the residual's mean removed first (as k_pcg_a/b).
// sE holds the level's padded cells compactly: (n0+2) x (n1+2) [x (n2+2)].
template <typename T, int D>
__device__ void bottom_pcg(const LevelRef<T>& v, int K, T* sE) {
  const Grid3& g = v.g;
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  const int m0 = g.n[0] + 2, m1 = g.n[1] + 2;
  const int lsz = m0 * m1 * ((D == 3) ? g.n[2] + 2 : 1);
  const int ls[3] = {1, m0, m0 * m1};
  // LDS offsets of the + and - neighbours, and their periodic-wrap forms
  int lp[3], lm[3], lpw[3], lmw[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lp[a] = ls[a];
    lm[a] = -ls[a];
    lpw[a] = -(g.n[a] - 1) * ls[a];
    lmw[a] = (g.n[a] - 1) * ls[a];
  }
  for (int i = threadIdx.x; i < lsz; i += kBottom) sE[i] = T(0);
  // this thread's cells (wrap: bit 2a for +a, bit 2a+1 for -a)
  bool ok[kBottomCPT];
  int gid[kBottomCPT], lid[kBottomCPT], wrap[kBottomCPT];
  T di[kBottomCPT], xr[kBottomCPT], rr[kBottomCPT], qq[kBottomCPT], ec[kBottomCPT];
  T Lp[kBottomCPT][3], Lm[kBottomCPT][3];
  double s = 0.0, c = 0.0;
#pragma unroll
  for (int k = 0; k < kBottomCPT; ++k) {
    const int lin = threadIdx.x + k * kBottom;
    ok[k] = lin < total;
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, ok[k] ? lin : 0, I, idx);
    nbr_offsets<D>(g, I, op, om);
    gid[k] = idx;
    lid[k] = I[0] + I[1] * ls[1] + ((D == 3) ? I[2] * ls[2] : 0);
    wrap[k] = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < D && g.per[a] && I[a] == g.n[a]) wrap[k] |= 1 << (2 * a);
      if (a < D && g.per[a] && I[a] == 1) wrap[k] |= 2 << (2 * a);
      Lp[k][a] = (a < D) ? v.L.c[a][idx + op[a]] : T(0);
      Lm[k][a] = (a < D) ? v.L.c[a][idx] : T(0);
    }
    di[k] = ok[k] ? v.iD[idx] : T(0);
    rr[k] = v.r[idx];
    xr[k] = v.x[idx];
    qq[k] = T(0);
    ec[k] = T(0);
    if (di[k] != T(0)) {
      s += double(rr[k]);
      c += 1.0;
    }
  }
  block_sum2<kBottom>(s, c);  // also orders the LDS clear before the first writes
  const T mean = T(c > 0.0 ? s / c : 0.0);
  double rho = 0.0, rho_prev = 0.0;
  for (int it = 0; it < K; ++it) {
    T beta = T(0);
    if (it > 0) {
      if (rho == 0.0) break;
      beta = T(rho / rho_prev);
    }
#pragma unroll
    for (int k = 0; k < kBottomCPT; ++k) {
      ec[k] = (it > 0) ? di[k] * rr[k] + beta * ec[k] : di[k] * (rr[k] - mean);
      if (ok[k]) sE[lid[k]] = ec[k];
    }
    __syncthreads();
    double sig = 0.0, r0 = 0.0;
#pragma unroll
    for (int k = 0; k < kBottomCPT; ++k) {
      T Ae = T(0);
      if (di[k] != T(0)) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const int op = ((wrap[k] >> (2 * a)) & 1) ? lpw[a] : lp[a];
          const int om = ((wrap[k] >> (2 * a)) & 2) ? lmw[a] : lm[a];
          Ae = Ae + Lp[k][a] * (sE[lid[k] + op] - ec[k]) - Lm[k][a] * (ec[k] - sE[lid[k] + om]);
        }
        if (it == 0) r0 += double(rr[k] - mean) * double(ec[k]);
      }
      qq[k] = Ae;
      sig += double(ec[k]) * double(Ae);
    }
    block_sum2<kBottom>(sig, r0);  // its barriers also end this sweep's LDS reads
    if (it == 0) rho = r0;
    if (fabs(sig) < 1e-300) break;
    const T alpha = T(rho / sig);
    double rn = 0.0;
#pragma unroll
    for (int k = 0; k < kBottomCPT; ++k) {
      T r_ = rr[k];
      if (it == 0 && di[k] != T(0)) r_ = r_ - mean;
      xr[k] = xr[k] + alpha * ec[k];
      r_ = r_ - alpha * qq[k];
      rr[k] = r_;
      rn += double(r_) * (double(di[k]) * double(r_));
    }
    rho_prev = rho;
    rho = block_sum<kBottom>(rn);
  }
#pragma unroll
  for (int k = 0; k < kBottomCPT; ++k)
    if (ok[k]) {
      v.x[gid[k]] = xr[k];
      v.r[gid[k]] = rr[k];
    }
  __syncthreads();
}

// residual restriction f -> c (sum of the children, 0 on solid coarse cells), x_c = 0
template <typename T, int D>
__device__ void bottom_restrict(const LevelRef<T>& f, const LevelRef<T>& c) {
  const int total = c.g.n[0] * c.g.n[1] * ((D == 3) ? c.g.n[2] : 1);
  for (int lin = threadIdx.x; lin < total; lin += kBottom) {
    int J[3], cidx;
    cell_of<D>(c.g, lin, J, cidx);
    const int base = (2 * J[0] - 1) + (2 * J[1] - 1) * f.g.s[1] + ((D == 3) ? (2 * J[2] - 1) * f.g.s[2] : 0);
    T sum = f.r[base] + f.r[base + 1] + f.r[base + f.g.s[1]] + f.r[base + 1 + f.g.s[1]];
    if (D == 3) {
      const int b2 = base + f.g.s[2];
      sum = sum + (f.r[b2] + f.r[b2 + 1] + f.r[b2 + f.g.s[1]] + f.r[b2 + 1 + f.g.s[1]]);
    }
    c.r[cidx] = (c.iD[cidx] != T(0)) ? sum : T(0);
    c.x[cidx] = T(0);
  }
  __syncthreads();
}

// prolongation c -> f: x_f += x_c[parent]; r_f -= A_f e with e the injected x_c
template <typename T, int D>
__device__ void bottom_prolong(const LevelRef<T>& f, const LevelRef<T>& c) {
  const int total = f.g.n[0] * f.g.n[1] * ((D == 3) ? f.g.n[2] : 1);
  for (int lin = threadIdx.x; lin < total; lin += kBottom) {
    int I[3], idx;
    cell_of<D>(f.g, lin, I, idx);
    const T ec = c.x[parent_idx<T, D>(c.g, I[0], I[1], I[2])];
    f.x[idx] = f.x[idx] + ec;
    if (f.iD[idx] != T(0)) {
      T Ae = T(0);
      for (int a = 0; a < D; ++a) {
        int Jp[3] = {I[0], I[1], I[2]}, Jm[3] = {I[0], I[1], I[2]};
        Jp[a] = wrapc(I[a] + 1, a, f.g);
        Jm[a] = wrapc(I[a] - 1, a, f.g);
        const T ep = c.x[parent_idx<T, D>(c.g, Jp[0], Jp[1], Jp[2])];
        const T em = c.x[parent_idx<T, D>(c.g, Jm[0], Jm[1], Jm[2])];
        const int op = (f.g.per[a] && I[a] == f.g.n[a]) ? -(f.g.n[a] - 1) * f.g.s[a] : f.g.s[a];
        Ae = Ae + f.L.c[a][idx + op] * (ep - ec) - f.L.c[a][idx] * (ec - em);
      }
      f.r[idx] = f.r[idx] - Ae;
    }
  }
  __syncthreads();
}

// The rest of the cycle from the first bottom level (whose residual the caller
// restricted): restrict down, PCG on the coarsest level, then prolong + PCG up.
// One block of kBottom threads.
template <typename T, int D>
__global__ void __launch_bounds__(kBottom) k_bottom(BottomLevels<T> bl) {
  __shared__ T sE[bottom_lds_elems<T>()];
  const int last = bl.n - 1;
  for (int l = 0; l < last; ++l) bottom_restrict<T, D>(bl.lv[l], bl.lv[l + 1]);
  bottom_pcg<T, D>(bl.lv[last], bl.pcg_iters, sE);
  for (int l = last - 1; l >= 0; --l) {
    bottom_prolong<T, D>(bl.lv[l], bl.lv[l + 1]);
    bottom_pcg<T, D>(bl.lv[l], bl.pcg_iters, sE);
  }
}

// ---------------------------------------------------------------------------
// Flat forms of the two PCG passes for a large 3-D level.  One thread per vector
// of W = 16 bytes / sizeof(T) consecutive interior cells along x (the rows must
// hold a whole number of vectors), consecutive threads along the rows, planes in
// order, so at any moment the whole GPU works on a narrow, contiguous window of
// each field.  The six neighbours come from the cache: the x neighbours are the
// vector's own lanes plus one scalar at each end, the y and z neighbours are the
// same-aligned vectors one row or one plane away, which neighbouring threads
// have just loaded.  Every thread runs once (no loop), so the loads of many
// short-lived waves overlap.  Each block leaves one FP64 partial per reduced
// quantity; a single-block kernel sums them (k_finalize2) before the next pass
// reads the total.
// ---------------------------------------------------------------------------
#ifndef WL_FLAT_THREADS
#define WL_FLAT_THREADS 256
#endif
constexpr int kFlatThreads = WL_FLAT_THREADS;
constexpr int kFinalizeThreads = 1024;
constexpr int kFinalizeStage = 128;  // blocks of the first stage of a two-stage total

// the thread's vector: first cell (i0, j, k), its field index, and whether it exists
struct FlatVec {
  int i0, j, k, id;
  bool ok;
};
template <typename T, bool REV = false>
__device__ __forceinline__ FlatVec flat_vec(const Grid3& g) {
  constexpr int W = Vec16<T>::W;
  // grid: x = the blocks of one plane, y = the plane (REV: the last block first)
  const unsigned vr = (unsigned)(g.n[0] / W);
  const unsigned bxx = REV ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
  const unsigned t = bxx * (unsigned)kFlatThreads + threadIdx.x;
  FlatVec f;
  f.ok = t < vr * (unsigned)g.n[1];
  const unsigned tt = f.ok ? t : 0u;
  const unsigned row = tt / vr;
  f.i0 = 1 + (int)(tt - row * vr) * W;
  f.j = (int)row + 1;
  f.k = (int)(REV ? gridDim.y - 1 - blockIdx.y : blockIdx.y) + 1;
  f.id = f.i0 + f.j * g.s[1] + f.k * g.s[2];
  return f;
}
// linear block index of a flat launch (its partial's slot)
__device__ __forceinline__ int flat_block() { return blockIdx.y * gridDim.x + blockIdx.x; }

// neighbour offsets of a vector (periodic wrap, else the ghost layer): x for the
// first lane's -x and the last lane's +x neighbour, y and z for the whole vector.
// PER = false: no periodic axis, so the offsets are constants.
template <int W, bool PER>
struct FlatNbr {
  int xm, xp, ym, yp, zm, zp;
  __device__ FlatNbr(const Grid3& g, const FlatVec& f) {
    xm = -1;
    xp = 1;
    ym = -g.s[1];
    yp = g.s[1];
    zm = -g.s[2];
    zp = g.s[2];
    if (PER) {
      if (g.per[0] && f.i0 == 1) xm = g.n[0] - 1;
      if (g.per[0] && f.i0 + W - 1 == g.n[0]) xp = -(g.n[0] - 1);
      if (g.per[1] && f.j == 1) ym = (g.n[1] - 1) * g.s[1];
      if (g.per[1] && f.j == g.n[1]) yp = -(g.n[1] - 1) * g.s[1];
      if (g.per[2] && f.k == 1) zm = (g.n[2] - 1) * g.s[2];
      if (g.per[2] && f.k == g.n[2]) zp = -(g.n[2] - 1) * g.s[2];
    }
  }
};

template <typename T>
__device__ __forceinline__ typename Vec16<T>::type ldv(const T* p) {
  return *reinterpret_cast<const typename Vec16<T>::type*>(p);
}
// a vector the kernel reads once and then overwrites (x and r of PCG pass B and of
// the prolongation, the fine residual of the restriction, u of the projection):
// a non-temporal load, which leaves the L2 to the vectors that neighbouring
// threads read again (the passes and the ones after them ran 2-20 % faster)
template <typename T>
__device__ __forceinline__ typename Vec16<T>::type ldv_stream(const T* p) {
  constexpr int W = Vec16<T>::W;
  typedef T NV __attribute__((ext_vector_type(W)));
  const NV n = __builtin_nontemporal_load(reinterpret_cast<const NV*>(p));
  typename Vec16<T>::type v;
  T* a = reinterpret_cast<T*>(&v);
#pragma unroll
  for (int w = 0; w < W; ++w) a[w] = n[w];
  return v;
}
template <typename T>
__device__ __forceinline__ void stv_stream(T* p, const typename Vec16<T>::type& v) {
  constexpr int W = Vec16<T>::W;
  const T* a = reinterpret_cast<const T*>(&v);
  typedef T NV __attribute__((ext_vector_type(W)));
  NV n;
#pragma unroll
  for (int w = 0; w < W; ++w) n[w] = a[w];
#if WL_NT_MODE >= 1
  __builtin_nontemporal_store(n, reinterpret_cast<NV*>(p));
#else
  *reinterpret_cast<NV*>(p) = n;
#endif
}

// is the vector's stencil (with the margin the tiles use) outside the body box?
template <int W>
__device__ __forceinline__ bool flat_fast(const StdBox& B, const Grid3& g, const FlatVec& f) {
  const int a[3] = {f.i0 - 2, f.j - 2, f.k - 2}, b[3] = {f.i0 + W + 1, f.j + 2, f.k + 2};
  return std_miss<3>(B, g, a, b);
}

// closed-form iD of a cell from the count of its non-periodic boundary faces
// (a chain of selects on thresholds: an equality chain is turned into an indexed
// table, which lives in scratch memory)
template <typename T>
__device__ __forceinline__ T std_iD_nb(const StdBox& B, int nb) {
  T r = std_iD<T>(B, 0);
  r = nb >= 1 ? std_iD<T>(B, 1) : r;
  r = nb >= 2 ? std_iD<T>(B, 2) : r;
  r = nb >= 3 ? std_iD<T>(B, 3) : r;
  return r;
}

// Coefficients of lane w of a vector: the inverse diagonal of its cell and the
// face coefficients at the cell and at its + neighbours.  Off the body box they
// are the closed form, evaluated without branches: the boundary faces of
// non-periodic axes carry 0 and a cell's iD depends on how many it has.  The
// vectors start at x = 1 and rows hold whole vectors, so only the first lane can
// touch the -x boundary and only the last the +x one; the y and z terms are the
// same for the whole vector.  Inside the box the coefficients are loaded.
template <typename T, int W, bool PER>
struct FlatStd {
  T Ls, Lyc, Lyp, Lzc, Lzp;
  int nbyz;
  bool x0, x1;
  __device__ __forceinline__ FlatStd(const Grid3& g, const StdBox& B, const FlatVec& f) {
    const bool px = PER && g.per[0], py = PER && g.per[1], pz = PER && g.per[2];
    Ls = T(B.Lstd);
    x0 = !px && f.i0 == 1;
    x1 = !px && f.i0 + W - 1 == g.n[0];
    const bool y0 = !py && f.j == 1, y1 = !py && f.j == g.n[1];
    const bool z0 = !pz && f.k == 1, z1 = !pz && f.k == g.n[2];
    nbyz = int(y0) + int(y1) + int(z0) + int(z1);
    Lyc = y0 ? T(0) : Ls;
    Lyp = y1 ? T(0) : Ls;
    Lzc = z0 ? T(0) : Ls;
    Lzp = z1 ? T(0) : Ls;
  }
  __device__ __forceinline__ bool xlo(int w) const { return w == 0 && x0; }
  __device__ __forceinline__ bool xhi(int w) const { return w == W - 1 && x1; }
  __device__ __forceinline__ T d(const StdBox& B, int w) const {
    return std_iD_nb<T>(B, nbyz + int(xlo(w)) + int(xhi(w)));
  }
};

// the coefficients of a vector near the body, loaded as whole vectors
template <typename T, int W, bool PER>
struct FlatLoaded {
  typename Vec16<T>::type d, lx, ly0, ly1, lz0, lz1;
  T lxe;  // x face past the last lane
  __device__ __forceinline__ FlatLoaded(const Grid3& g, const Vec3<T>& L, const T* iD, const FlatVec& f,
                                        const FlatNbr<W, PER>& o) {
    const int id = f.id;
    d = ldv(iD + id);
    lx = ldv(L.c[0] + id);
    lxe = L.c[0][id + W - 1 + ((PER && g.per[0] && f.i0 + W - 1 == g.n[0]) ? -(g.n[0] - 1) : 1)];
    ly0 = ldv(L.c[1] + id);
    ly1 = ldv(L.c[1] + id + o.yp);
    lz0 = ldv(L.c[2] + id);
    lz1 = ldv(L.c[2] + id + o.zp);
  }
};

template <typename T, int W, bool PER>
struct FlatCoef {
  T d, Lxp, Lxc, Lyp, Lyc, Lzp, Lzc;
  // closed form
  __device__ __forceinline__ FlatCoef(const FlatStd<T, W, PER>& S, const StdBox& B, int w) {
    d = S.d(B, w);
    Lxc = S.xlo(w) ? T(0) : S.Ls;
    Lxp = S.xhi(w) ? T(0) : S.Ls;
    Lyc = S.Lyc;
    Lyp = S.Lyp;
    Lzc = S.Lzc;
    Lzp = S.Lzp;
  }
  // loaded
  __device__ __forceinline__ FlatCoef(const FlatLoaded<T, W, PER>& C, int w) {
    const T* D = reinterpret_cast<const T*>(&C.d);
    const T* LX = reinterpret_cast<const T*>(&C.lx);
    d = D[w];
    Lxc = LX[w];
    Lxp = (w < W - 1) ? LX[w + 1] : C.lxe;
    Lyc = reinterpret_cast<const T*>(&C.ly0)[w];
    Lyp = reinterpret_cast<const T*>(&C.ly1)[w];
    Lzc = reinterpret_cast<const T*>(&C.lz0)[w];
    Lzp = reinterpret_cast<const T*>(&C.lz1)[w];
  }
};

// e_new of one cell: iD r + beta e_old (sweep 0: iD (r - m)).  One function, so a
// cell recomputed as a neighbour gets the value its own thread stores.
template <typename T>
__device__ __forceinline__ T pcg_e(T d, T r, T e, T beta, T mean, int k) {
  return (k > 0) ? d * r + beta * e : d * (r - mean);
}

// (FINE = 1 only makes the fine-level launches of the flat kernels separate
// symbols in kernel traces.)
// PCG pass A, flat form (arithmetic of k_pcg_a_tile with STOREQ = 0): e_new of
// the vector (stored) and of its -x, -y and -z neighbour cells (recomputed from
// their r, e_old and iD), the sigma = e.Ae partial and, in sweep 0, the rho_0
// partial.  sigma is summed over faces: A holds the face coefficients off the
// diagonal and minus their sum on it, so e.Ae = -sum over faces of
// L_f (e_i - e_j)^2; each cell takes its three - faces (a periodic axis wraps
// face 1 to cell N; a non-periodic boundary face has L = 0, and a solid cell,
// iD = 0, has only zero faces).
// (FP32: at least 8 waves per SIMD, 61 registers without spills, 1 % faster
// than the 66 the compiler picks by itself)
template <typename T, bool PER, int FINE>
__global__ void __launch_bounds__(kFlatThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1)))
k_pcg_a_fused_flat(Grid3 g, Vec3<T> L, const T* iD, const T* r,
                                                                   const T* eo, T* en, double* red, int k, RedN rn,
                                                                   double* part_sig, double* part_rho0, int* flag,
                                                                   StdBox B) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  if (*flag) return;
  T beta, mean;
  if (!pcg_a_scalars<T, kFlatThreads>(red, k, rn, flag, beta, mean)) return;
  const FlatVec f = flat_vec<T>(g);
  double sig = 0.0, rho0 = 0.0;
  if (f.ok) {
    const FlatNbr<W, PER> o(g, f);
    const int id = f.id;
    // grid-uniform branch on k: sweep 0 reads no e_old
    V r0 = ldv(r + id), ry = ldv(r + id + o.ym), rz = ldv(r + id + o.zm), e0 = {}, ey = {}, ez = {};
    const T rx = r[id + o.xm];
    T ex = T(0);
    if (k > 0) {
      e0 = ldv(eo + id);
      ey = ldv(eo + id + o.ym);
      ez = ldv(eo + id + o.zm);
      ex = eo[id + o.xm];
    }
    const T *R0 = reinterpret_cast<const T*>(&r0), *RY = reinterpret_cast<const T*>(&ry),
            *RZ = reinterpret_cast<const T*>(&rz);
    const T *E0 = reinterpret_cast<const T*>(&e0), *EY = reinterpret_cast<const T*>(&ey),
            *EZ = reinterpret_cast<const T*>(&ez);
    T d[W], dy[W], dz[W], dx, lx[W], ly[W], lz[W];
    if (flat_fast<W>(B, g, f)) {
      // closed form; a neighbour cell's iD counts its own non-periodic boundary faces
      const bool py = PER && g.per[1], pz = PER && g.per[2];
      const FlatStd<T, W, PER> S(g, B, f);
      const int cy = int(!py && f.j == 1) + int(!py && f.j == g.n[1]);
      const int cz = int(!pz && f.k == 1) + int(!pz && f.k == g.n[2]);
      const int cym = int(!py && f.j - 1 == 1) + int(!py && f.j - 1 == g.n[1]);
      const int czm = int(!pz && f.k - 1 == 1) + int(!pz && f.k - 1 == g.n[2]);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int cx = int(S.xlo(w)) + int(S.xhi(w));
        d[w] = std_iD_nb<T>(B, cx + cy + cz);
        dy[w] = std_iD_nb<T>(B, cx + cym + cz);
        dz[w] = std_iD_nb<T>(B, cx + cy + czm);
        lx[w] = S.xlo(w) ? T(0) : S.Ls;
        ly[w] = S.Lyc;
        lz[w] = S.Lzc;
      }
      // the -x neighbour of the first lane is interior in x, or the wrapped last
      // cell of a periodic row (a non-periodic boundary face has L = 0)
      dx = std_iD_nb<T>(B, cy + cz);
    } else {
      const V d0 = ldv(iD + id), dyv = ldv(iD + id + o.ym), dzv = ldv(iD + id + o.zm);
      const V lxv = ldv(L.c[0] + id), lyv = ldv(L.c[1] + id), lzv = ldv(L.c[2] + id);
      dx = iD[id + o.xm];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        d[w] = reinterpret_cast<const T*>(&d0)[w];
        dy[w] = reinterpret_cast<const T*>(&dyv)[w];
        dz[w] = reinterpret_cast<const T*>(&dzv)[w];
        lx[w] = reinterpret_cast<const T*>(&lxv)[w];
        ly[w] = reinterpret_cast<const T*>(&lyv)[w];
        lz[w] = reinterpret_cast<const T*>(&lzv)[w];
      }
    }
    V out;
    T* O = reinterpret_cast<T*>(&out);
    T prev = pcg_e<T>(dx, rx, ex, beta, mean, k);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const T ec = pcg_e<T>(d[w], R0[w], E0[w], beta, mean, k);
      const T eym = pcg_e<T>(dy[w], RY[w], EY[w], beta, mean, k);
      const T ezm = pcg_e<T>(dz[w], RZ[w], EZ[w], beta, mean, k);
      O[w] = ec;
      // a zero face adds nothing (and its neighbour may be a ghost cell)
      const T jx = lx[w] != T(0) ? ec - prev : T(0), jy = ly[w] != T(0) ? ec - eym : T(0),
              jz = lz[w] != T(0) ? ec - ezm : T(0);
      sig -= double(lx[w] * (jx * jx) + ly[w] * (jy * jy) + lz[w] * (jz * jz));
      if (k == 0 && d[w] != T(0)) rho0 += double(R0[w] - mean) * double(ec);
      prev = ec;
    }
    stv_stream<T>(en + id, out);
  }
  sig = block_sum<kFlatThreads>(sig);
  if (threadIdx.x == 0) part_sig[flat_block()] = sig;
  if (k == 0) {
    rho0 = block_sum<kFlatThreads>(rho0);
    if (threadIdx.x == 0) part_rho0[flat_block()] = rho0;
  }
}

// Sum of r^2 over the interior cells (FP64), flat form: one 16-byte vector of
// cells per thread, the block's sum into part.
template <typename T>
__global__ void __launch_bounds__(kFlatThreads) k_sumsq_flat(Grid3 g, const T* r, double* part) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  const FlatVec f = flat_vec<T>(g);
  double s = 0.0;
  if (f.ok) {
    const V rv = ldv(r + f.id);
    const T* R = reinterpret_cast<const T*>(&rv);
#pragma unroll
    for (int w = 0; w < W; ++w) s += double(R[w]) * double(R[w]);
  }
  s = block_sum<kFlatThreads>(s);
  if (threadIdx.x == 0) part[flat_block()] = s;
}

// CFL and divergence check, flat form (arithmetic of k_cfl): one 16-byte vector
// of cells per thread; per cell sigma = sum_a max(0, u_a[I + e_a]) + max(0,
// -u_a[I]) and div = sum_a (u_a[I + e_a] - u_a[I]) in FP64, the block's maxima of
// sigma and of |div| over the active cells into part / part_div.
template <typename T, bool PER>
__global__ void __launch_bounds__(kFlatThreads) k_cfl_flat(Grid3 g, Vec3<T> u, const T* iD, StdBox B,
                                                           double* part, double* part_div) {
#pragma clang fp contract(off)
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  const FlatVec f = flat_vec<T>(g);
  double mx = 0.0, md = 0.0;
  if (f.ok) {
    const FlatNbr<W, PER> o(g, f);
    const int id = f.id;
    const V u0 = ldv(u.c[0] + id), u1 = ldv(u.c[1] + id), u1p = ldv(u.c[1] + id + o.yp), u2 = ldv(u.c[2] + id),
            u2p = ldv(u.c[2] + id + o.zp);
    const T u0n = u.c[0][id + W - 1 + o.xp];
    // cells of the vector outside the body box are active; inside, those with iD != 0
    const int a[3] = {f.i0, f.j, f.k}, b[3] = {f.i0 + W - 1, f.j, f.k};
    const bool all_act = std_miss<3>(B, g, a, b);
    V dv_ = {};
    if (!all_act) dv_ = ldv(iD + id);
    const T *U0 = reinterpret_cast<const T*>(&u0), *U1 = reinterpret_cast<const T*>(&u1),
            *U1P = reinterpret_cast<const T*>(&u1p), *U2 = reinterpret_cast<const T*>(&u2),
            *U2P = reinterpret_cast<const T*>(&u2p), *DI = reinterpret_cast<const T*>(&dv_);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const T up0 = (w < W - 1) ? U0[w + 1] : u0n;
      T s = T(0);
      s = s + fmax(T(0), up0) + fmax(T(0), -U0[w]);
      s = s + fmax(T(0), U1P[w]) + fmax(T(0), -U1[w]);
      s = s + fmax(T(0), U2P[w]) + fmax(T(0), -U2[w]);
      double dv = 0.0;
      dv = dv + (double(up0) - double(U0[w]));
      dv = dv + (double(U1P[w]) - double(U1[w]));
      dv = dv + (double(U2P[w]) - double(U2[w]));
      mx = fmax(mx, double(s));
      bool act = all_act;
      if (!act) {
        const int I[3] = {f.i0 + w, f.j, f.k};
        act = std_point<3>(B, g, I, 0) || DI[w] != T(0);
      }
      if (act) md = fmax(md, fabs(dv));
    }
  }
  mx = block_max<kFlatThreads>(mx);
  md = block_max<kFlatThreads>(md);
  if (threadIdx.x == 0) {
    part[flat_block()] = mx;
    part_div[flat_block()] = md;
  }
}

// PCG pass B, flat form (arithmetic of k_pcg_b_tile): q = A e from e and its
// neighbours, x += alpha e, r -= alpha q, partials of rho_{k+1} and max|r|.
template <typename T, bool PER, int FINE>
__global__ void __launch_bounds__(kFlatThreads) k_pcg_b_flat(Grid3 g, Vec3<T> L, const T* iD, const T* e, T* x,
                                                             T* r, double* red, int k, RedN rn,
                                                             double* part_rho_next, double* part_max, int want_rho,
                                                             int want_max, int* flag, StdBox B) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  // the blocks in reverse order (the last vectors first): this pass and the pass A
  // after it ran 0.5-0.8 % faster than with both in the same order
  const FlatVec f = flat_vec<T, true>(g);
  // the stream loads go out first; the stop flag and the scalars are read while
  // they are in flight
  V ec_ = {}, ey0 = {}, ey1 = {}, ez0 = {}, ez1 = {}, xv = {}, rv = {};
  T ex0 = T(0), ex1 = T(0);
  if (f.ok) {
    const FlatNbr<W, PER> o(g, f);
    const int id = f.id;
    ec_ = ldv(e + id);
    ey0 = ldv(e + id + o.ym);
    ey1 = ldv(e + id + o.yp);
    ez0 = ldv(e + id + o.zm);
    ez1 = ldv(e + id + o.zp);
    ex0 = e[id + o.xm];
    ex1 = e[id + W - 1 + o.xp];
    xv = ldv_stream<T>(x + id);
    rv = ldv_stream<T>(r + id);
  }
  bool skip = (*flag) != 0;
  T alpha = T(0);
  const T mean = (k == 0) ? T(residual_mean<kFlatThreads>(red, rn.mean)) : T(0);
  if (!skip) {
    const double sig = total_of<kFlatThreads>(red + (size_t)(kSlotSig0 + k) * kMaxBlocks, rn.sig);
    if (fabs(sig) < 1e-300) {
      skip = true;
      if (flat_block() == 0 && threadIdx.x == 0) *flag = 1;
    } else {
      alpha = T(total_of<kFlatThreads>(red + (size_t)(kSlotRho0 + k) * kMaxBlocks, rn.rho) / sig);
    }
  }
  if (skip && !want_max && mean == T(0)) return;  // grid-uniform
  double rho = 0.0, mx = 0.0;
  if (f.ok) {
    const FlatNbr<W, PER> o(g, f);
    const int id = f.id;
    const T* E0 = reinterpret_cast<const T*>(&ec_);
    const T *EY0 = reinterpret_cast<const T*>(&ey0), *EY1 = reinterpret_cast<const T*>(&ey1);
    const T *EZ0 = reinterpret_cast<const T*>(&ez0), *EZ1 = reinterpret_cast<const T*>(&ez1);
    const T* X0 = reinterpret_cast<const T*>(&xv);
    const T* R0 = reinterpret_cast<const T*>(&rv);
    V xo, ro;
    T* XO = reinterpret_cast<T*>(&xo);
    T* RO = reinterpret_cast<T*>(&ro);
    auto lane = [&](const FlatCoef<T, W, PER>& c, int w) {
      const T ec = E0[w];
      T rr = R0[w];
      if (mean != T(0) && c.d != T(0)) rr = rr - mean;
      XO[w] = X0[w];
      if (!skip) {
        T qq = T(0);
        if (c.d != T(0)) {
          const T xm = (w > 0) ? E0[w - 1] : ex0, xp = (w < W - 1) ? E0[w + 1] : ex1;
          qq = qq + c.Lxp * (xp - ec) - c.Lxc * (ec - xm);
          qq = qq + c.Lyp * (EY1[w] - ec) - c.Lyc * (ec - EY0[w]);
          qq = qq + c.Lzp * (EZ1[w] - ec) - c.Lzc * (ec - EZ0[w]);
        }
        XO[w] = X0[w] + alpha * ec;
        rr = rr - alpha * qq;
      }
      RO[w] = rr;
      rho += double(rr) * (double(c.d) * double(rr));
      mx = fmax(mx, fabs(double(rr)));
    };
    if (flat_fast<W>(B, g, f)) {
      const FlatStd<T, W, PER> S(g, B, f);
#pragma unroll
      for (int w = 0; w < W; ++w) lane(FlatCoef<T, W, PER>(S, B, w), w);
    } else {
      const FlatLoaded<T, W, PER> C(g, L, iD, f, o);
#pragma unroll
      for (int w = 0; w < W; ++w) lane(FlatCoef<T, W, PER>(C, w), w);
    }
    if (!skip) stv_stream<T>(x + id, xo);
    if (!skip || mean != T(0)) stv_stream<T>(r + id, ro);
  }
  if ((want_rho && !skip) || want_max) {
    // one exchange for both: the sum of rho and the max of |r|
    __shared__ double shr[kFlatThreads / 64], shm[kFlatThreads / 64];
    rho = wave_sum(rho);
    mx = wave_max(mx);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
      shr[wv] = rho;
      shm[wv] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double sr = shr[0], sm = shm[0];
#pragma unroll
      for (int i = 1; i < kFlatThreads / 64; ++i) {
        sr += shr[i];
        sm = fmax(sm, shm[i]);
      }
      if (want_rho && !skip) part_rho_next[flat_block()] = sr;
      if (want_max) part_max[flat_block()] = sm;
    }
  }
}

// Divergence (or a given right-hand side), warm start and initial residual,
// flat form (arithmetic of k_div_res): x = p wdt (if p) else the current x,
// r = z - A x on active cells (0 elsewhere); partials of max|r| and of the mean
// of r over the active cells.
template <typename T, bool PER>
__global__ void __launch_bounds__(kFlatThreads) k_div_res_flat(Grid3 g, Vec3<T> u, const T* rhs, const T* p, T wdt,
                                                               Vec3<T> L, const T* iD, T* x, T* r, double* part_max,
                                                               double* part_sum, double* part_cnt, int* flag,
                                                               StdBox B) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  if (flat_block() == 0 && threadIdx.x == 0) *flag = 0;
  const FlatVec fv = flat_vec<T>(g);
  double mx = 0.0, sr = 0.0, cnt = 0.0;
  if (fv.ok) {
    const FlatNbr<W, PER> o(g, fv);
    const int id = fv.id;
    const T* xs = p ? p : x;
    const T sx = p ? wdt : T(1);
    const V xv = ldv(xs + id), xy0 = ldv(xs + id + o.ym), xy1 = ldv(xs + id + o.yp), xz0 = ldv(xs + id + o.zm),
            xz1 = ldv(xs + id + o.zp);
    const T xm0 = xs[id + o.xm] * sx, xp0 = xs[id + W - 1 + o.xp] * sx;
    V zv;
    T* Z = reinterpret_cast<T*>(&zv);
    if (rhs) {
      zv = ldv(rhs + id);
    } else {
      const V ux = ldv(u.c[0] + id), uy = ldv(u.c[1] + id), uy1 = ldv(u.c[1] + id + o.yp), uz = ldv(u.c[2] + id),
              uz1 = ldv(u.c[2] + id + o.zp);
      const T ux1 = u.c[0][id + W - 1 + o.xp];
      const T* UX = reinterpret_cast<const T*>(&ux);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const T uxp = (w < W - 1) ? UX[w + 1] : ux1;
        T z = T(0);
        z = z + (uxp - UX[w]);
        z = z + (reinterpret_cast<const T*>(&uy1)[w] - reinterpret_cast<const T*>(&uy)[w]);
        z = z + (reinterpret_cast<const T*>(&uz1)[w] - reinterpret_cast<const T*>(&uz)[w]);
        Z[w] = z;
      }
    }
    T xc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) xc[w] = reinterpret_cast<const T*>(&xv)[w] * sx;
    V ro, xo;
    T* RO = reinterpret_cast<T*>(&ro);
    T* XO = reinterpret_cast<T*>(&xo);
    auto lane = [&](const FlatCoef<T, W, PER>& cf, int w) {
      T rr = T(0);
      if (cf.d != T(0)) {
        const T xm = (w > 0) ? xc[w - 1] : xm0, xp = (w < W - 1) ? xc[w + 1] : xp0;
        const T ym = reinterpret_cast<const T*>(&xy0)[w] * sx, yp = reinterpret_cast<const T*>(&xy1)[w] * sx;
        const T zm = reinterpret_cast<const T*>(&xz0)[w] * sx, zp = reinterpret_cast<const T*>(&xz1)[w] * sx;
        T Ax = T(0);
        Ax = Ax + cf.Lxp * (xp - xc[w]) - cf.Lxc * (xc[w] - xm);
        Ax = Ax + cf.Lyp * (yp - xc[w]) - cf.Lyc * (xc[w] - ym);
        Ax = Ax + cf.Lzp * (zp - xc[w]) - cf.Lzc * (xc[w] - zm);
        rr = Z[w] - Ax;
        sr += double(rr);
        cnt += 1.0;
      }
      RO[w] = rr;
      XO[w] = xc[w];
      mx = fmax(mx, fabs(double(rr)));
    };
    if (flat_fast<W>(B, g, fv)) {
      const FlatStd<T, W, PER> S(g, B, fv);
#pragma unroll
      for (int w = 0; w < W; ++w) lane(FlatCoef<T, W, PER>(S, B, w), w);
    } else {
      const FlatLoaded<T, W, PER> C(g, L, iD, fv, o);
#pragma unroll
      for (int w = 0; w < W; ++w) lane(FlatCoef<T, W, PER>(C, w), w);
    }
    if (p) stv_stream<T>(x + id, xo);
    stv_stream<T>(r + id, ro);
  }
  sr = block_sum<kFlatThreads>(sr);
  cnt = block_sum<kFlatThreads>(cnt);
  mx = block_max<kFlatThreads>(mx);
  if (threadIdx.x == 0) {
    part_max[flat_block()] = mx;
    part_sum[flat_block()] = sr;
    part_cnt[flat_block()] = cnt;
  }
}

// Projection update, flat form (arithmetic of k_project): u_a -= L_a (x[I] -
// x[I-e_a]) on the interior faces of each vector, p = x / wdt.
template <typename T, bool PER>
__global__ void __launch_bounds__(kFlatThreads) k_project_flat(Grid3 g, Vec3<T> u, Vec3<T> L, const T* x, T* p,
                                                               T wdt, StdBox B) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  const FlatVec fv = flat_vec<T>(g);
  if (!fv.ok) return;  // no barrier in this kernel
  const FlatNbr<W, PER> o(g, fv);
  const int id = fv.id;
  const V xv = ldv(x + id), xy = ldv(x + id + o.ym), xz = ldv(x + id + o.zm);
  const T xm0 = x[id + o.xm];
  V u0 = ldv_stream<T>(u.c[0] + id), u1 = ldv_stream<T>(u.c[1] + id), u2 = ldv_stream<T>(u.c[2] + id);
  const int a[3] = {fv.i0, fv.j, fv.k}, b[3] = {fv.i0 + W - 1, fv.j, fv.k};
  const bool fast = std_miss<3>(B, g, a, b);
  V l0, l1, l2;
  if (!fast) {
    l0 = ldv(L.c[0] + id);
    l1 = ldv(L.c[1] + id);
    l2 = ldv(L.c[2] + id);
  }
  const T* X = reinterpret_cast<const T*>(&xv);
  const T* XY = reinterpret_cast<const T*>(&xy);
  const T* XZ = reinterpret_cast<const T*>(&xz);
  T* U0 = reinterpret_cast<T*>(&u0);
  T* U1 = reinterpret_cast<T*>(&u1);
  T* U2 = reinterpret_cast<T*>(&u2);
  V pv;
  T* PV = reinterpret_cast<T*>(&pv);
  const T Ly = L_std<T>(g, B, 1, fv.j), Lz = L_std<T>(g, B, 2, fv.k);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const T xc = X[w];
    const T xmx = (w > 0) ? X[w - 1] : xm0;
    const T L0 = fast ? L_std<T>(g, B, 0, fv.i0 + w) : reinterpret_cast<const T*>(&l0)[w];
    const T L1 = fast ? Ly : reinterpret_cast<const T*>(&l1)[w];
    const T L2 = fast ? Lz : reinterpret_cast<const T*>(&l2)[w];
    U0[w] = U0[w] - L0 * (xc - xmx);
    U1[w] = U1[w] - L1 * (xc - XY[w]);
    U2[w] = U2[w] - L2 * (xc - XZ[w]);
    PV[w] = xc / wdt;
  }
  stv_stream<T>(u.c[0] + id, u0);
  stv_stream<T>(u.c[1] + id, u1);
  stv_stream<T>(u.c[2] + id, u2);
  if (p) stv_stream<T>(p + id, pv);
}

// BDIM blend, flat form (arithmetic of k_bdim) over the padded faces of one
// component (blockIdx.z) and plane (blockIdx.y).  The first threads of a plane
// take the vectors of x-faces 1..N of every padded row: those whose faces all lie
// outside the body box take the closed form (u = L f, or u = f with no body)
// with vector loads and stores, the others near the body the blend with vector
// loads, or face by face next to the domain boundary.  The last 2 (N_y + 2)
// threads take the x ghost faces 0 and N + 1 of each row, so no wave of vectors
// also runs the per-face path.
template <typename T, int CORR>
__global__ void __launch_bounds__(kFlatThreads) k_bdim_flat(Grid3 g, Vec3<T> f, Vec3<T> V, Vec3<T> mu0,
                                                            Vec9<T> mu1, Vec3<T> u, int has_body, StdBox B) {
  typedef typename Vec16<T>::type VT;
  constexpr int W = Vec16<T>::W;
  const int c = blockIdx.z;
  const int vr = g.n[0] / W;  // vectors of a row: first cells 1, 1 + W, ...
  const int P1 = g.n[1] + 2;
  const int t = blockIdx.x * kFlatThreads + threadIdx.x;
  const int k = blockIdx.y;
  if (t >= vr * P1) {
    const int e = t - vr * P1;
    if (e >= 2 * P1) return;  // no barrier in this kernel
    const int I[3] = {(e & 1) ? g.n[0] + 1 : 0, e >> 1, k};
    bdim_face<T, 3, CORR>(g, f, V, mu0, mu1, u, has_body, B, c, I, lin3<T, 3>(g, I[0], I[1], I[2]), u);
    return;
  }
  const int m = t % vr, j = t / vr;
  const int i0 = 1 + m * W;
  const int id = i0 + j * g.s[1] + k * g.s[2];
  bool fastv = true;
  if (has_body) {
    const int a[3] = {i0, j, k}, b[3] = {i0 + W - 1, j, k};
    fastv = std_miss<3>(B, g, a, b);
  }
  if (fastv) {
    const VT fv = ldv(f.c[c] + id);
    VT uv;
    if (CORR) uv = ldv(u.c[c] + id);
    const T* F = reinterpret_cast<const T*>(&fv);
    T* U = reinterpret_cast<T*>(&uv);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int Ic = (c == 0) ? i0 + w : (c == 1 ? j : k);
      const T acc = has_body ? L_std<T>(g, B, c, Ic) * F[w] : F[w];
      U[w] = CORR ? T(0.5) * (U[w] + acc) : acc;
    }
    stv_stream<T>(u.c[c] + id, uv);
  } else if (i0 >= 2 && i0 + W - 1 <= g.n[0] - 1 && j >= 2 && j <= g.n[1] - 1 && k >= 2 &&
             k <= g.n[2] - 1) {
    // near the body, away from the domain boundary: the blend of bdim_face with
    // whole-vector loads of f, V, mu0, mu1 (the x neighbours of f from the lanes)
    const T* fc = f.c[c];
    const VT fv = ldv(fc + id), fy0 = ldv(fc + id - g.s[1]), fy1 = ldv(fc + id + g.s[1]),
             fz0 = ldv(fc + id - g.s[2]), fz1 = ldv(fc + id + g.s[2]);
    const T fx0 = fc[id - 1], fx1 = fc[id + W];
    const VT vv = ldv(V.c[c] + id), m0 = ldv(mu0.c[c] + id), mx = ldv(mu1.c[c * 3] + id),
             my = ldv(mu1.c[c * 3 + 1] + id), mz = ldv(mu1.c[c * 3 + 2] + id);
    VT uv;
    if (CORR) uv = ldv(u.c[c] + id);
    const T* F = reinterpret_cast<const T*>(&fv);
    T* U = reinterpret_cast<T*>(&uv);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const T xm = (w > 0) ? F[w - 1] : fx0, xp = (w < W - 1) ? F[w + 1] : fx1;
      T acc = reinterpret_cast<const T*>(&vv)[w] + reinterpret_cast<const T*>(&m0)[w] * F[w];
      acc = acc + reinterpret_cast<const T*>(&mx)[w] * (T(0.5) * (xp - xm));
      acc = acc + reinterpret_cast<const T*>(&my)[w] *
                      (T(0.5) * (reinterpret_cast<const T*>(&fy1)[w] - reinterpret_cast<const T*>(&fy0)[w]));
      acc = acc + reinterpret_cast<const T*>(&mz)[w] *
                      (T(0.5) * (reinterpret_cast<const T*>(&fz1)[w] - reinterpret_cast<const T*>(&fz0)[w]));
      U[w] = CORR ? T(0.5) * (U[w] + acc) : acc;
    }
    stv_stream<T>(u.c[c] + id, uv);
  } else {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int I[3] = {i0 + w, j, k};
      bdim_face<T, 3, CORR>(g, f, V, mu0, mu1, u, has_body, B, c, I, id + w, u);
    }
  }
}

// Residual restriction, flat form (arithmetic of k_restrict): one thread per
// vector of W coarse cells, whose 2 x 2 x 2 children are two fine vectors in each
// of two rows of two planes (the vectors of both levels start at odd x).  r_c is
// the children's sum on active coarse cells (0 elsewhere), x_c = 0, and the
// partials of the mean of r_c.
template <typename T, bool PER, int FINE>
__global__ void __launch_bounds__(kFlatThreads) k_restrict_flat(Grid3 f, Grid3 c, const T* rf, const T* iDc, T* rc,
                                                                T* xc, double* part_sum, double* part_cnt, int* flag,
                                                                StdBox Bc) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  if (flat_block() == 0 && threadIdx.x == 0) *flag = 0;
  const FlatVec cv = flat_vec<T>(c);
  double sr = 0.0, cnt = 0.0;
  if (cv.ok) {
    const int fb = (2 * cv.i0 - 1) + (2 * cv.j - 1) * f.s[1] + (2 * cv.k - 1) * f.s[2];
    const int s1 = f.s[1], s2 = f.s[2];
    // rows (y, z) = (0,0), (1,0), (0,1), (1,1); two vectors each
    const V a0 = ldv_stream<T>(rf + fb), a1 = ldv_stream<T>(rf + fb + W), b0 = ldv_stream<T>(rf + fb + s1),
            b1 = ldv_stream<T>(rf + fb + s1 + W);
    const V c0 = ldv_stream<T>(rf + fb + s2), c1 = ldv_stream<T>(rf + fb + s2 + W),
            d0 = ldv_stream<T>(rf + fb + s2 + s1), d1 = ldv_stream<T>(rf + fb + s2 + s1 + W);
    auto at = [](const V& lo, const V& hi, int q) -> T {
      return q < W ? reinterpret_cast<const T*>(&lo)[q] : reinterpret_cast<const T*>(&hi)[q - W];
    };
    V ro, xo;
    T* RO = reinterpret_cast<T*>(&ro);
    T* XO = reinterpret_cast<T*>(&xo);
    const bool fast = flat_fast<W>(Bc, c, cv);
    V dl;
    if (!fast) dl = ldv(iDc + cv.id);
    const FlatStd<T, W, PER> S(c, Bc, cv);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int q = 2 * w;
      T sm = at(a0, a1, q) + at(a0, a1, q + 1) + at(b0, b1, q) + at(b0, b1, q + 1);
      sm = sm + (at(c0, c1, q) + at(c0, c1, q + 1) + at(d0, d1, q) + at(d0, d1, q + 1));
      const T di = fast ? S.d(Bc, w) : reinterpret_cast<const T*>(&dl)[w];
      RO[w] = (di != T(0)) ? sm : T(0);
      XO[w] = T(0);
      if (di != T(0)) {
        sr += double(RO[w]);
        cnt += 1.0;
      }
    }
    stv_stream<T>(rc + cv.id, ro);
    stv_stream<T>(xc + cv.id, xo);
  }
  sr = block_sum<kFlatThreads>(sr);
  cnt = block_sum<kFlatThreads>(cnt);
  if (threadIdx.x == 0) {
    part_sum[flat_block()] = sr;
    part_cnt[flat_block()] = cnt;
  }
}

// Prolongation + correction, flat form (arithmetic of k_prolong): e = x_c of the
// parent, x += e, and on active cells r -= A e; partials of the mean of the new
// r.  With the vectors starting at odd x, lanes 2h and 2h+1 share the coarse
// parent h; the other parents the stencil reaches are the x neighbours of the
// end lanes and one coarse row and plane beside (whichever of j - 1, j + 1 and
// k - 1, k + 1 leaves the parent's row or plane).
template <typename T, bool PER, int FINE>
__global__ void __launch_bounds__(kFlatThreads) k_prolong_flat(Grid3 f, Grid3 c, const T* xc, Vec3<T> L,
                                                               const T* iD, T* xf, T* rf, double* part_sum,
                                                               double* part_cnt, int* flag, StdBox B) {
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W, H = W / 2;
  if (flat_block() == 0 && threadIdx.x == 0) *flag = 0;
  const FlatVec fv = flat_vec<T>(f);
  double sr = 0.0, cnt = 0.0;
  if (fv.ok) {
    const FlatNbr<W, PER> o(f, fv);
    const int id = fv.id;
    const V xv = ldv_stream<T>(xf + id), rv = ldv_stream<T>(rf + id);
    const int Ic0 = (fv.i0 + 1) >> 1, J = (fv.j + 1) >> 1, K = (fv.k + 1) >> 1;
    const int im = (PER && f.per[0] && fv.i0 == 1) ? f.n[0] : fv.i0 - 1;
    const int ip = (PER && f.per[0] && fv.i0 + W - 1 == f.n[0]) ? 1 : fv.i0 + W;
    const bool jodd = (fv.j & 1) != 0, kodd = (fv.k & 1) != 0;
    int jn = jodd ? fv.j - 1 : fv.j + 1, kn = kodd ? fv.k - 1 : fv.k + 1;
    if (PER && f.per[1]) jn = wrapc(jn, 1, f);
    if (PER && f.per[2]) kn = wrapc(kn, 2, f);
    const int Jo = (jn + 1) >> 1, Ko = (kn + 1) >> 1;
    const int row = J * c.s[1] + K * c.s[2];
    T ec[H], ey[H], ez[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      ec[h] = xc[Ic0 + h + row];
      ey[h] = xc[Ic0 + h + Jo * c.s[1] + K * c.s[2]];
      ez[h] = xc[Ic0 + h + J * c.s[1] + Ko * c.s[2]];
    }
    const T ecm = xc[((im + 1) >> 1) + row], ecp = xc[((ip + 1) >> 1) + row];
    const T* X0 = reinterpret_cast<const T*>(&xv);
    const T* R0 = reinterpret_cast<const T*>(&rv);
    V xo, ro;
    T* XO = reinterpret_cast<T*>(&xo);
    T* RO = reinterpret_cast<T*>(&ro);
    auto lane = [&](const FlatCoef<T, W, PER>& cf, int w) {
      const T e0 = ec[w >> 1];
      XO[w] = X0[w] + e0;
      T rr = R0[w];
      if (cf.d != T(0)) {
        const T xm = (w == 0) ? ecm : ec[(w - 1) >> 1], xp = (w == W - 1) ? ecp : ec[(w + 1) >> 1];
        const T ym = jodd ? ey[w >> 1] : e0, yp = jodd ? e0 : ey[w >> 1];
        const T zm = kodd ? ez[w >> 1] : e0, zp = kodd ? e0 : ez[w >> 1];
        T Ae = T(0);
        Ae = Ae + cf.Lxp * (xp - e0) - cf.Lxc * (e0 - xm);
        Ae = Ae + cf.Lyp * (yp - e0) - cf.Lyc * (e0 - ym);
        Ae = Ae + cf.Lzp * (zp - e0) - cf.Lzc * (e0 - zm);
        rr = rr - Ae;
        sr += double(rr);
        cnt += 1.0;
      }
      RO[w] = rr;
    };
    if (flat_fast<W>(B, f, fv)) {
      const FlatStd<T, W, PER> S(f, B, fv);
#pragma unroll
      for (int w = 0; w < W; ++w) lane(FlatCoef<T, W, PER>(S, B, w), w);
    } else {
      const FlatLoaded<T, W, PER> C(f, L, iD, fv, o);
#pragma unroll
      for (int w = 0; w < W; ++w) lane(FlatCoef<T, W, PER>(C, w), w);
    }
    stv_stream<T>(xf + id, xo);
    stv_stream<T>(rf + id, ro);
  }
  sr = block_sum<kFlatThreads>(sr);
  cnt = block_sum<kFlatThreads>(cnt);
  if (threadIdx.x == 0) {
    part_sum[flat_block()] = sr;
    part_cnt[flat_block()] = cnt;
  }
}

// out_a[b] = sum (or max, a_max) of block b's share of a[0..n), out_b[b] likewise
// for b; either array may be NULL.  One block gives the total; G blocks leave G
// partials.  Fixed order, so repeated runs agree bitwise.
__global__ void __launch_bounds__(kFinalizeThreads) k_finalize2(const double* a, int a_max, const double* b,
                                                                int b_max, int n, double* out_a, double* out_b) {
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double sa = 0.0, sb = 0.0;
  // four loads in flight per thread and trip: a single block then sums ~16 k
  // partials in a few memory round trips
  constexpr int U = 4;
  for (int i0 = lo + threadIdx.x; i0 < hi; i0 += U * kFinalizeThreads) {
    double va[U], vb[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = i0 + q * kFinalizeThreads;
      const bool in = i < hi;
      va[q] = (a && in) ? a[i] : 0.0;
      vb[q] = (b && in) ? b[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (i0 + q * kFinalizeThreads >= hi) break;
      if (a) sa = a_max ? fmax(sa, va[q]) : sa + va[q];
      if (b) sb = b_max ? fmax(sb, vb[q]) : sb + vb[q];
    }
  }
  if (a) sa = a_max ? block_max<kFinalizeThreads>(sa) : block_sum<kFinalizeThreads>(sa);
  if (b) sb = b_max ? block_max<kFinalizeThreads>(sb) : block_sum<kFinalizeThreads>(sb);
  if (threadIdx.x == 0) {
    if (a) out_a[blockIdx.x] = sa;
    if (b) out_b[blockIdx.x] = sb;
  }
}

// single-block max / sum of partials into a scalar slot
__global__ void __launch_bounds__(kBlock) k_finalize_max(const double* part, int n, double* out) {
  const double v = max_of(part, n);
  if (threadIdx.x == 0) *out = v;
}

// projection update u_a -= L_a (x[I] - x[I-e_a]) on interior cells; p = x / wdt.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_project(Grid3 g, Vec3<T> u, Vec3<T> L, const T* x, T* p, T wdt,
                                                    StdBox B) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, lin, I, idx);
    nbr_offsets<D>(g, I, op, om);
    const T xc = x[idx];
    const bool sc = std_point<D>(B, g, I, 0);
    for (int a = 0; a < D; ++a) {
      const T Lc = sc ? L_std<T>(g, B, a, I[a]) : L.c[a][idx];
      u.c[a][idx] = u.c[a][idx] - Lc * (xc - x[idx + om[a]]);
    }
    if (p) p[idx] = xc / wdt;
  }
}

// CFL: max over interior cells of sum_a max(0, u_a[I+e_a]) + max(0, -u_a[I]), and
// the projection check max |div u| over the active cells (iD != 0), the
// divergence summed in FP64.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_cfl(Grid3 g, Vec3<T> u, const T* iD, StdBox B, double* part,
                                                double* part_div) {
#pragma clang fp contract(off)
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double mx = 0.0, md = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, lin, I, idx);
    nbr_offsets<D>(g, I, op, om);
    T s = T(0);
    double dv = 0.0;
    for (int a = 0; a < D; ++a) {
      const T up = u.c[a][idx + op[a]], uc = u.c[a][idx];
      s = s + fmax(T(0), up) + fmax(T(0), -uc);
      dv = dv + (double(up) - double(uc));
    }
    mx = fmax(mx, double(s));
    const bool act = std_point<D>(B, g, I, 0) || iD[idx] != T(0);
    if (act) md = fmax(md, fabs(dv));
  }
  mx = block_max(mx);
  md = block_max(md);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = mx;
    part_div[blockIdx.x] = md;
  }
}

// Sum of r^2 over the interior cells (FP64): blocks take whole rows, threads
// stride along x.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_sumsq(Grid3 g, const T* r, double* part) {
  const int rows = g.n[1] * ((D == 3) ? g.n[2] : 1);
  double s = 0.0;
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int j = 1 + row % g.n[1], k = (D == 3) ? 1 + row / g.n[1] : 0;
    const T* rr = r + j * g.s[1] + k * g.s[2];
    for (int i = 1 + threadIdx.x; i <= g.n[0]; i += kBlock) {
      const double v = double(rr[i]);
      s += v * v;
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// forces: F_p = -sum (p - pbar) n K_eps(d), F_v = sum 2 nu S n K_eps(d) at cell centres
// (FP64), pbar = mean of p over active cells.  Partials: sum p n K, sum 2 nu S n K,
// sum n K, sum_active p, active count; the host combines them.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_forces(Grid3 g, BodyP b, Motion m, double eps, double nu,
                                                   Vec3<T> u, const T* p, const T* iD, double* part,
                                                   int stride) {
#pragma clang fp contract(off)
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double fp[3] = {0, 0, 0}, fv[3] = {0, 0, 0}, nk[3] = {0, 0, 0}, ps = 0.0, pc = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    if (iD[idx] != T(0)) {
      ps += double(p[idx]);
      pc += 1.0;
    }
    double x[3] = {I[0] - 0.5, I[1] - 0.5, I[2] - 0.5}, d, n[3], V[3];
    body_eval<D>(b, m, x, d, n, V);
    const double w = kern_K(d, eps);
    if (w == 0.0) continue;
    const double pv = double(p[idx]);
    for (int a = 0; a < D; ++a) {
      fp[a] += pv * n[a] * w;
      nk[a] += n[a] * w;
    }
    // velocity gradient G[i][j] = d u_i / d x_j at the cell centre
    double G[3][3];
    for (int i = 0; i < D; ++i) {
      const T* ui = u.c[i];
      const int si = g.s[i];
      for (int j = 0; j < D; ++j) {
        if (j == i) {
          G[i][j] = double(ui[idx + si]) - double(ui[idx]);
        } else {
          const int sj = g.s[j];
          const double bp = 0.5 * (double(ui[idx + sj]) + double(ui[idx + sj + si]));
          const double bm = 0.5 * (double(ui[idx - sj]) + double(ui[idx - sj + si]));
          G[i][j] = 0.5 * (bp - bm);
        }
      }
    }
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int j = 0; j < D; ++j) acc = acc + 0.5 * (G[i][j] + G[j][i]) * n[j];
      fv[i] += 2.0 * nu * acc * w;
    }
  }
  for (int a = 0; a < 3; ++a) {
    const double sp = block_sum(fp[a]);
    const double sv = block_sum(fv[a]);
    const double sn = block_sum(nk[a]);
    if (threadIdx.x == 0) {
      part[(size_t)a * stride + blockIdx.x] = sp;
      part[(size_t)(3 + a) * stride + blockIdx.x] = sv;
      part[(size_t)(6 + a) * stride + blockIdx.x] = sn;
    }
  }
  ps = block_sum(ps);
  pc = block_sum(pc);
  if (threadIdx.x == 0) {
    part[(size_t)9 * stride + blockIdx.x] = ps;
    part[(size_t)10 * stride + blockIdx.x] = pc;
  }
}

// Totals of rows of partials: block r sums part[r * stride + 0 .. n-1] into out[r]
// (fixed order: strided per thread, then the block tree).
__global__ void __launch_bounds__(kBlock) k_sum_rows(const double* part, int n, int stride, double* out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) v += part[(size_t)blockIdx.x * stride + i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* a, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) a[i] = v;
}

}  // namespace wl

// Discrete adjoint of the BDIM predictor-corrector step: one transpose kernel per
// forward kernel (numerical-methods section; the paper itself differentiates the
// solver in forward mode with dual numbers, this is the reverse-mode counterpart).
//
// Conventions: the time step is frozen; the limiter is linearised on the branch
// the forward took (a tie picks the first argument in median order); the
// multigrid solve counts as the exact solution operator of A x = P z on the active
// cells (P removes the mean over active cells), whose transpose is P A^+ P since
// A is symmetric.  Bars denote adjoints.  Scatter-form transposes accumulate with
// global atomics, so results are reproducible to rounding, not bitwise.
#pragma once
#include "wl_kernels.hpp"

namespace wl {

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  atomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// boundary conditions.  The forward rule, axis k = 0 .. D-1 in turn over the
// full padded extent of the other axes: periodic k copies u[0] = u[N],
// u[N+1] = u[1]; the component's own non-periodic axis prescribes faces 0, 1,
// N+1; a tangential non-periodic axis copies u[0] = u[1], u[N+1] = u[N].
// Transpose: axes D-1 .. 0, ghost adjoints moved onto their sources and zeroed,
// prescribed adjoints zeroed.  One launch per axis, blockIdx.y = component; a
// thread owns a whole line along the axis.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_bc_axis(Grid3 g, Vec3<T> ub, int k) {
  const int c = blockIdx.y;
  T* const w = ub.c[c];
  const int o0 = (k == 0) ? 1 : 0, o1 = (k == 2) ? 1 : 2;
  const int m0 = g.n[o0] + 2, m1 = (D == 3) ? g.n[o1] + 2 : 1;
  const int N = g.n[k];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < m0 * m1; lin += gridDim.x * kBlock) {
    int I[3] = {0, 0, 0};
    I[o0] = lin % m0;
    if (D == 3) I[o1] = lin / m0;
    const int base = I[0] + I[1] * g.s[1] + I[2] * g.s[2];
    const int sk = g.s[k];
    T* const l0 = w + base;  // I_k = 0
    if (g.per[k]) {
      l0[sk] = l0[sk] + l0[(N + 1) * sk];
      l0[N * sk] = l0[N * sk] + l0[0];
      l0[(N + 1) * sk] = T(0);
      l0[0] = T(0);
    } else if (k == c) {
      l0[0] = T(0);
      l0[sk] = T(0);
      l0[(N + 1) * sk] = T(0);
    } else {
      l0[sk] = l0[sk] + l0[0];
      l0[N * sk] = l0[N * sk] + l0[(N + 1) * sk];
      l0[0] = T(0);
      l0[(N + 1) * sk] = T(0);
    }
  }
}

// ---------------------------------------------------------------------------
// projection with weight w: z = Dv u (all interior cells), A x = P z on active
// cells, u_a[I] -= L_a[I] (x[I] - x[I-e_a]) for interior cells I, p = x / (w dt).
//   xbar  = pbar/(w dt) - G^T (L ubar)          (active cells; 0 elsewhere)
//   lam   = P A^+ P xbar                         (multigrid solve + mean removal)
//   ubar += Dv^T lam ;  Lbar_a[I] -= (x[I] - x[I-e_a]) ubar_a[I]   (after the update)
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_proj_rhs(Grid3 g, Vec3<T> ub, Vec3<T> L, const T* pb, T inv_wdt,
                                                         const T* iD, T* rhs) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, lin, I, idx);
    nbr_offsets<D>(g, I, op, om);
    T v = T(0);
    if (iD[idx] != T(0)) {
      if (pb) v = pb[idx] * inv_wdt;
      // the forward update of face I+e_a uses x[I] with +L, that of face I with -L;
      // L vanishes on non-periodic boundary faces
      for (int a = 0; a < D; ++a) v = v - (L.c[a][idx] * ub.c[a][idx] - L.c[a][idx + op[a]] * ub.c[a][idx + op[a]]);
    }
    rhs[idx] = v;
  }
}

// Faces of component a = blockIdx.y: J_a in 1..N_a (periodic) or 1..N_a+1, other
// axes interior.  lam is mean-removed over active cells with the sum/count
// partials of the last mean producer (nparts blocks).  Lbar accumulates into Lb.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_proj_update(Grid3 g, Vec3<T> ub, const T* lam, const T* x,
                                                            const T* iD, Vec3<T> Lb, const double* red,
                                                            int nparts) {
  const int a = blockIdx.y;
  const double mean = residual_mean(red, nparts);
  const bool per = g.per[a] != 0;
  int m[3];
  for (int k = 0; k < 3; ++k) m[k] = (k < D) ? (g.n[k] + ((k == a && !per) ? 1 : 0)) : 1;
  const int total = m[0] * m[1] * m[2];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int J[3];
    J[0] = lin % m[0] + 1;
    const int t = lin / m[0];
    J[1] = t % m[1] + 1;
    J[2] = (D == 3) ? t / m[1] + 1 : 0;
    const int idx = J[0] + J[1] * g.s[1] + J[2] * g.s[2];
    const int jm = per ? wrapc(J[a] - 1, a, g) : J[a] - 1;
    const int im = idx + (jm - J[a]) * g.s[a];
    const bool own = J[a] <= g.n[a];  // cell J exists (face N+1 of a non-periodic axis has none)
    const bool low = jm >= 1;         // cell J - e_a exists
    const T lc = (own && iD[idx] != T(0)) ? T(double(lam[idx]) - mean) : T(0);
    const T lm = (low && iD[im] != T(0)) ? T(double(lam[im]) - mean) : T(0);
    const T u = ub.c[a][idx] + (lm - lc);
    ub.c[a][idx] = u;
    // the forward velocity update (faces 1..N) used L; on non-periodic boundary faces L is 0
    if (own && low) Lb.c[a][idx] = Lb.c[a][idx] - (x[idx] - x[im]) * u;
  }
}

// ---------------------------------------------------------------------------
// BDIM blend out = V + mu0 f + sum_j mu1_cj (f[I+e_j] - f[I-e_j])/2 on every padded
// face (the wrap and validity of the forward), u = out (predictor) or
// u = (u + out)/2 (corrector).  With w = s ubar (s = 1 or 1/2):
//   fbar  = mu0 w + M1^T w      (gather; assigned)
//   Vbar += w,  mu0bar += w f,  mu1bar_cj += w (f[+j] - f[-j])/2
//   corrector: ubar_prev = ubar/2 (assigned to up).
// The gather reads w at the faces whose stencil touches this one; on a periodic
// axis those are taken among interior faces only, which is exact because the
// boundary-condition transpose leaves a zero adjoint on every ghost face.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bdim_pair_ok(const Grid3& g, int Ij, int j) {
  return g.per[j] || (Ij + 1 <= g.n[j] + 1 && Ij - 1 >= 0);
}

template <typename T, int D, int CORR>
__global__ void __launch_bounds__(kBlock) k_adj_bdim(Grid3 g, Vec3<T> ub, Vec3<T> f, Vec3<T> mu0, Vec9<T> mu1,
                                                     Vec3<T> fb, Vec3<T> Vb, Vec3<T> mu0b, Vec9<T> mu1b, Vec3<T> up,
                                                     int has_body) {
  const int c = blockIdx.y;
  const T s = CORR ? T(0.5) : T(1);
  const int P0 = g.n[0] + 2, P1 = g.n[1] + 2, P2 = (D == 3) ? g.n[2] + 2 : 1;
  const int total = P0 * P1 * P2;
  const T* const uc = ub.c[c];
  const T* const fc = f.c[c];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I[3] = {lin % P0, (lin / P0) % P1, (D == 3) ? lin / (P0 * P1) : 0};
    const int idx = I[0] + I[1] * g.s[1] + I[2] * g.s[2];
    const T w = s * uc[idx];
    if (CORR) up.c[c][idx] = w;
    if (!has_body) {
      fb.c[c][idx] = w;
      continue;
    }
    T acc = mu0.c[c][idx] * w;
    for (int j = 0; j < D; ++j) {
      const int sj = g.s[j], N = g.n[j];
      const T* const m1 = mu1.c[c * D + j];
      // face I is the +j neighbour of I - e_j and the -j neighbour of I + e_j
      if (g.per[j]) {
        if (I[j] >= 1 && I[j] <= N) {
          const int lo = (I[j] == 1) ? idx + (N - 1) * sj : idx - sj;
          const int hi = (I[j] == N) ? idx - (N - 1) * sj : idx + sj;
          acc = acc + T(0.5) * m1[lo] * (s * uc[lo]) - T(0.5) * m1[hi] * (s * uc[hi]);
        }
      } else {
        if (I[j] - 1 >= 0 && bdim_pair_ok(g, I[j] - 1, j)) acc = acc + T(0.5) * m1[idx - sj] * (s * uc[idx - sj]);
        if (I[j] + 1 <= N + 1 && bdim_pair_ok(g, I[j] + 1, j)) acc = acc - T(0.5) * m1[idx + sj] * (s * uc[idx + sj]);
      }
      // mu1 adjoint with the forward's neighbour pair
      if (bdim_pair_ok(g, I[j], j)) {
        int ip = idx + sj, im = idx - sj;
        if (g.per[j]) {
          ip = idx + (wrapc(I[j] + 1, j, g) - I[j]) * sj;
          im = idx + (wrapc(I[j] - 1, j, g) - I[j]) * sj;
        }
        mu1b.c[c * D + j][idx] = mu1b.c[c * D + j][idx] + w * (T(0.5) * (fc[ip] - fc[im]));
      }
    }
    fb.c[c][idx] = acc;
    Vb.c[c][idx] = Vb.c[c][idx] + w;
    mu0b.c[c][idx] = mu0b.c[c][idx] + w * fc[idx];
  }
}

// ---------------------------------------------------------------------------
// convection-diffusion: f~ = u0 + dt R(u) - V (every padded face; R only on the
// unknown faces).  u0bar += fbar and Vbar -= fbar everywhere; ubar += dt R'(u)^T fbar
// by scattering each flux's linearisation (atomics).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int median_arg(T a, T b, T c) {
  const T m = median3(a, b, c);
  return (m == a) ? 0 : ((m == b) ? 1 : 2);
}

// gv = dJ/dPhi_cj at (wrapped) index J; scatter d Phi / d u into ub
template <typename T, int D>
__device__ __forceinline__ void adj_phi(const Grid3& g, const Vec3<T>& u, const Vec3<T>& ub, int c, int j,
                                        const int J[3], T nu, T gv) {
  int Jc[3] = {J[0], J[1], J[2]};
  Jc[c] = wrapc(J[c] - 1, c, g);
  int Jj[3] = {J[0], J[1], J[2]};
  Jj[j] = wrapc(J[j] - 1, j, g);
  const int iJ = lin3<T, D>(g, J[0], J[1], J[2]);
  const int iJc = lin3<T, D>(g, Jc[0], Jc[1], Jc[2]);
  const int iJj = lin3<T, D>(g, Jj[0], Jj[1], Jj[2]);
  const T a = T(0.5) * (u.c[j][iJ] + u.c[j][iJc]);
  const T uc = u.c[c][iJ];
  const T m1 = u.c[c][iJj];
  const bool upw = a >= T(0);
  int F[3] = {J[0], J[1], J[2]};
  const int fx = upw ? J[j] - 2 : J[j] + 1;
  bool ok;
  if (g.per[j]) {
    F[j] = wrapc(fx, j, g);
    ok = true;
  } else {
    F[j] = fx;
    ok = fx >= 1 && fx <= (j == c ? g.n[j] + 1 : g.n[j]);
  }
  T Q, duc, dm1, dfar = T(0);
  int iF = 0;
  if (ok) {
    iF = lin3<T, D>(g, F[0], F[1], F[2]);
    const T far = u.c[c][iF];
    const T cc = upw ? m1 : uc, dd = upw ? uc : m1;  // (far, c, d) of the upwind triple
    const T q = (T(5) * cc + T(2) * dd - far) * T(1.0 / 6.0);  // as in quick_lim (same branch)
    const T ex = cc + T(9) * (cc - far);
    const T inner = median3(cc, dd, ex);
    Q = median3(cc, q, inner);
    T gc = T(0), gd = T(0), gf = T(0);
    const int o = median_arg(cc, q, inner);
    if (o == 0) {
      gc = T(1);
    } else if (o == 1) {
      gc = T(5) / T(6);
      gd = T(2) / T(6);
      gf = T(-1) / T(6);
    } else {
      const int i2 = median_arg(cc, dd, ex);
      if (i2 == 0) {
        gc = T(1);
      } else if (i2 == 1) {
        gd = T(1);
      } else {
        gc = T(10);
        gf = T(-9);
      }
    }
    dfar = gf;
    duc = upw ? gd : gc;
    dm1 = upw ? gc : gd;
  } else {
    Q = T(0.5) * (uc + m1);
    duc = T(0.5);
    dm1 = T(0.5);
  }
  // Phi = a Q - nu (uc - m1)
  const T ga = gv * Q * T(0.5);
  atomic_add(&ub.c[j][iJ], ga);
  atomic_add(&ub.c[j][iJc], ga);
  const T gq = gv * a;
  if (ok) atomic_add(&ub.c[c][iF], gq * dfar);
  atomic_add(&ub.c[c][iJ], gq * duc - gv * nu);
  atomic_add(&ub.c[c][iJj], gq * dm1 + gv * nu);
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_flux(Grid3 g, Vec3<T> u, Vec3<T> fb, Vec3<T> ub, Vec3<T> u0b,
                                                     Vec3<T> Vb, T dt, T nu, int has_body) {
  const int c = blockIdx.y;
  const int P0 = g.n[0] + 2, P1 = g.n[1] + 2, P2 = (D == 3) ? g.n[2] + 2 : 1;
  const int total = P0 * P1 * P2;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I[3] = {lin % P0, (lin / P0) % P1, (D == 3) ? lin / (P0 * P1) : 0};
    const int idx = lin3<T, D>(g, I[0], I[1], I[2]);
    const T f = fb.c[c][idx];
    atomic_add(&u0b.c[c][idx], f);
    if (has_body) Vb.c[c][idx] = Vb.c[c][idx] - f;
    bool unknown = true;
    for (int a = 0; a < D; ++a) {
      const int lo = (a == c && !g.per[a]) ? 2 : 1;
      unknown = unknown && I[a] >= lo && I[a] <= g.n[a];
    }
    const T Rb = dt * f;
    if (!unknown || Rb == T(0)) continue;
    for (int j = 0; j < D; ++j) {
      int Jp[3] = {I[0], I[1], I[2]};
      Jp[j] = wrapc(I[j] + 1, j, g);
      adj_phi<T, D>(g, u, ub, c, j, I, nu, Rb);
      adj_phi<T, D>(g, u, ub, c, j, Jp, nu, -Rb);
    }
  }
}

// ---------------------------------------------------------------------------
// force functional g * dir . (F_p + F_v) at cell centres (FP64):
//   F_p = -sum (p - pbar) n K,  F_v = sum 2 nu S n K,  pbar = mean of p over active cells.
// Pressure adjoint: pbar_adj += -g (dir.n K - [active] dir.nkm), nkm = (sum n K)/count.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_force_p(Grid3 g, BodyP b, Motion m, double eps, const T* iD,
                                                        double gcoef, double3 dir, double nkm_dot, T* pb) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    double x[3] = {I[0] - 0.5, I[1] - 0.5, I[2] - 0.5}, d, n[3], V[3];
    body_eval<D>(b, m, x, d, n, V);
    const double K = kern_K(d, eps);
    const double dn = dir.x * n[0] + dir.y * n[1] + (D == 3 ? dir.z * n[2] : 0.0);
    double v = dn * K;
    if (iD[idx] != T(0)) v -= nkm_dot;
    pb[idx] = pb[idx] + T(-gcoef * v);
  }
}

// Viscous adjoint scattered into ub; per-block partials of the direct derivative
// with respect to the sphere radius through K(d), d = |x - P| - R (part[block]).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_force_v(Grid3 g, BodyP b, Motion m, double eps, double nu,
                                                        double gcoef, double3 dir, Vec3<T> u, const T* p, double pbar,
                                                        Vec3<T> ub, double* part) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  const double dv[3] = {dir.x, dir.y, dir.z};
  double dR = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    double x[3] = {I[0] - 0.5, I[1] - 0.5, I[2] - 0.5}, d, n[3], V[3];
    body_eval<D>(b, m, x, d, n, V);
    const double s = d / eps;
    if (!(fabs(s) < 1.0)) continue;
    const double K = 0.5 * (1.0 + cos(M_PI * s)) / eps;
    const double dKdd = -0.5 * M_PI * sin(M_PI * s) / (eps * eps);
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
    double integrand = 0.0, dn = 0.0;
    for (int i = 0; i < D; ++i) {
      double Sn = 0.0;
      for (int j = 0; j < D; ++j) Sn += 0.5 * (G[i][j] + G[j][i]) * n[j];
      integrand += dv[i] * (2.0 * nu * Sn);
      dn += dv[i] * n[i];
    }
    integrand -= (double(p[idx]) - pbar) * dn;
    if (b.p[0].kind == kShapeSphere) dR -= gcoef * integrand * dKdd;  // dd/dR = -1
    // dF/dG_ij = nu K (dir_i n_j + dir_j n_i)
    for (int i = 0; i < D; ++i) {
      const int si = g.s[i];
      for (int j = 0; j < D; ++j) {
        const double Gb = gcoef * nu * K * (dv[i] * n[j] + dv[j] * n[i]);
        if (Gb == 0.0) continue;
        if (j == i) {
          atomic_add(&ub.c[i][idx + si], T(Gb));
          atomic_add(&ub.c[i][idx], T(-Gb));
        } else {
          const int sj = g.s[j];
          const T q = T(0.25 * Gb);
          atomic_add(&ub.c[i][idx + sj], q);
          atomic_add(&ub.c[i][idx + sj + si], q);
          atomic_add(&ub.c[i][idx - sj], -q);
          atomic_add(&ub.c[i][idx - sj + si], -q);
        }
      }
    }
  }
  dR = block_sum(dR);
  if (threadIdx.x == 0) part[blockIdx.x] = dR;
}

// ---------------------------------------------------------------------------
// body parameters of a sphere/circle whose shape does not move (spin allowed):
//   d mu0/dR = -K_eps(d) (faces that measure does not force to 0),
//   d mu1_cj/dR = s K(s) n_j (s = d/eps; 0 where the solid cut zeroes mu1),
//   d V/d omega = (e_z x r)_c where V is set (d < 2 + eps).
// Partials (blockIdx.y = component): part[c*G + bx] = dJ/dR, part[(3+c)*G + bx] = dJ/domega.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_body(Grid3 g, BodyP b, Motion m, double eps, Vec3<T> mu0b,
                                                     Vec9<T> mu1b, Vec3<T> Vb, double* part) {
  const int c = blockIdx.y;
  const int P0 = g.n[0] + 2, P1 = g.n[1] + 2, P2 = (D == 3) ? g.n[2] + 2 : 1;
  const int total = P0 * P1 * P2;
  double dR = 0.0, dW = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I[3] = {lin % P0, (lin / P0) % P1, (D == 3) ? lin / (P0 * P1) : 0};
    const int idx = I[0] + I[1] * g.s[1] + I[2] * g.s[2];
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = (a == c) ? I[a] - 1.0 : I[a] - 0.5;
    double d, n[3], V[3];
    body_eval<D>(b, m, x, d, n, V);
    const double s = d / eps;
    if (fabs(s) < 1.0 && kern_mu0(d, eps) >= kMu0Cut) {
      const double Ks = 0.5 * (1.0 + cos(M_PI * s));
      const bool bnd = !g.per[c] && (I[c] <= 1 || I[c] == g.n[c] + 1);
      if (!bnd) dR -= double(mu0b.c[c][idx]) * Ks / eps;
      for (int j = 0; j < D; ++j) dR += double(mu1b.c[c * D + j][idx]) * s * Ks * n[j];
    }
    if (d < 2.0 + eps) {
      const double rx = x[0] - m.m[0].P[0], ry = x[1] - m.m[0].P[1];
      const double ezr = (c == 0) ? -ry : ((c == 1) ? rx : 0.0);
      dW += double(Vb.c[c][idx]) * ezr;
    }
  }
  dR = block_sum(dR);
  dW = block_sum(dW);
  if (threadIdx.x == 0) {
    part[c * gridDim.x + blockIdx.x] = dR;
    part[(3 + c) * gridDim.x + blockIdx.x] = dW;
  }
}

// ---------------------------------------------------------------------------
// Time-step derivative (steps whose dt follows the CFL rule).  Within one step
// dt enters through f~ = u0 + dt R - V in both stages and through p = x / (w dt)
// after the corrector (w = 1/2), so
//   dtbar = [<fbar_1, f~_1 - u0 + V> + <fbar_2, f~_2 - u0 + V>] / dt - <pbar, p> / dt,
// and dt_n = 1 / (sigma(I*) + 5 nu) of the state u^n, I* the cell of the largest
// outflux sigma = sum_a max(0, u_a[I+e_a]) + max(0, -u_a[I]) (the first such cell
// in x-fastest order), adds dtbar (-dt^2) d sigma(I*)/du to ubar of u^n.
// ---------------------------------------------------------------------------
// per-block partials of the sum over padded faces of fb . (f - u0 + V)
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_dt_flux(Grid3 g, Vec3<T> fb, Vec3<T> f, Vec3<T> u0, Vec3<T> V,
                                                        double* part) {
  const int P0 = g.n[0] + 2, P1 = g.n[1] + 2, P2 = (D == 3) ? g.n[2] + 2 : 1;
  const int total = P0 * P1 * P2;
  double s = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int I0 = lin % P0, I1 = (lin / P0) % P1, I2 = (D == 3) ? lin / (P0 * P1) : 0;
    const int idx = I0 + I1 * g.s[1] + I2 * g.s[2];
    for (int c = 0; c < D; ++c) {
      const double dR = double(f.c[c][idx]) - double(u0.c[c][idx]) + double(V.c[c][idx]);
      s += double(fb.c[c][idx]) * dR;
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// per-block partials of the sum over interior cells of pb p
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_dt_press(Grid3 g, const T* pb, const T* p, double* part) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double s = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    s += double(pb[idx]) * double(p[idx]);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// larger (v, i) pair: the larger value, on equal values the smaller index
__device__ __forceinline__ bool arg_better(double v, double i, double bv, double bi) {
  return v > bv || (v == bv && i < bi);
}

// per-block largest outflux over interior cells and its cell (linear index, x fastest)
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_cfl_arg(Grid3 g, Vec3<T> u, double* part_v, double* part_i) {
  const int total = g.n[0] * g.n[1] * ((D == 3) ? g.n[2] : 1);
  double bv = -1.0, bi = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx, op[3], om[3];
    cell_of<D>(g, lin, I, idx);
    nbr_offsets<D>(g, I, op, om);
    T s = T(0);
    for (int a = 0; a < D; ++a) s = s + fmax(T(0), u.c[a][idx + op[a]]) + fmax(T(0), -u.c[a][idx]);
    if (arg_better(double(s), double(lin), bv, bi)) {
      bv = double(s);
      bi = double(lin);
    }
  }
  __shared__ double sv[kBlock], si[kBlock];
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h && arg_better(sv[threadIdx.x + h], si[threadIdx.x + h], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + h];
      si[threadIdx.x] = si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_v[blockIdx.x] = sv[0];
    part_i[blockIdx.x] = si[0];
  }
}

// One block: the argmax cell from the partials, then ubar += c d sigma/du at it
// (c = dtbar (-dt^2)).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adj_cfl(Grid3 g, Vec3<T> u, Vec3<T> ub, const double* part_v,
                                                    const double* part_i, int n, double c) {
  double bv = -1.0, bi = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock)
    if (arg_better(part_v[k], part_i[k], bv, bi)) {
      bv = part_v[k];
      bi = part_i[k];
    }
  __shared__ double sv[kBlock], si[kBlock];
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h && arg_better(sv[threadIdx.x + h], si[threadIdx.x + h], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + h];
      si[threadIdx.x] = si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  int I[3], idx, op[3], om[3];
  cell_of<D>(g, (int)si[0], I, idx);
  nbr_offsets<D>(g, I, op, om);
  for (int a = 0; a < D; ++a) {
    if (u.c[a][idx + op[a]] > T(0)) ub.c[a][idx + op[a]] += T(c);
    if (-u.c[a][idx] > T(0)) ub.c[a][idx] -= T(c);
  }
}

}  // namespace wl

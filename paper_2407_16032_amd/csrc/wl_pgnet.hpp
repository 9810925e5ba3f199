// Learned multigrid initial guess: BF16 conv-net kernels (MFMA, FP32 accumulate).
//
// The net maps [p_{m-1}, p_{m-2}, z_m] (normalised) to the pressure change of the
// next solve: conv3^3(3->16)+ReLU, conv3^3(16->16)+ReLU, conv3^3(16->1).  Every
// convolution is an implicit GEMM on v_mfma_f32_16x16x16_bf16: a wave takes 16
// consecutive x-points of one row (M = 16), and each 3x3x3 tap is one 16x16x16
// product of (points x input channels) by (input channels x output channels).
// Activations are channels-last bfloat16 on a box with a one-cell zero halo.
#pragma once
#include "wl_device.hpp"

namespace wl {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPgHidden = 16;
constexpr int kPgCrop = 64;  // training crop interior (cells per axis)
// flat FP32 parameter vector: W1[27][3][16] b1[16] W2[27][16][16] b2[16] W3[27][16][1] b3[1]
constexpr int kPgW1 = 0, kPgB1 = kPgW1 + 27 * 3 * 16, kPgW2 = kPgB1 + 16, kPgB2 = kPgW2 + 27 * 16 * 16,
              kPgW3 = kPgB2 + 16, kPgB3 = kPgW3 + 27 * 16, kPgParams = kPgB3 + 1;

// A box of points with a one-cell zero halo: interior 1..n, padded dims n+2.
struct PgBox {
  int n[3];
  int P[3];  // n + 2
};

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ int pg_pt(const PgBox& b, int x, int y, int z) { return (z * b.P[1] + y) * b.P[0] + x; }

// Convolution on a box.  CIN = 4 (3 real channels) or 16; weights wf[27][CIN][16]
// in bfloat16, 16 output channels (unused ones carry zero weights).
// MODE 0: out = bf16(ReLU(acc + bias))              (hidden layer, forward)
// MODE 1: outf[p] = acc[channel 0] + bias[0]        (output layer, FP32)
// MODE 2: out = bf16(acc) where ref > 0, else 0     (backward data through a ReLU)
template <int CIN, int MODE>
__global__ void __launch_bounds__(kBlock) k_pg_conv(PgBox b, const unsigned short* in, const unsigned short* wf,
                                                    const float* bias, unsigned short* out, float* outf,
                                                    const unsigned short* ref) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  // B operands (weights) for all taps in registers: lane holds B[k = 4 lg + v][j = li]
  constexpr int NB = (CIN == 16) ? 27 : 7;
  bf16x4 bw[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (CIN == 16) {
        bw[q][v] = (short)wf[(q * 16 + 4 * lg + v) * 16 + li];
      } else {
        const int tap = 4 * q + lg;
        bw[q][v] = (tap < 27) ? (short)wf[(tap * 4 + v) * 16 + li] : (short)0;
      }
    }
  }
  const float bj = (MODE == 2) ? 0.f : bias[li];
  const int nxc = (b.n[0] + 15) / 16;
  const int ntask = nxc * b.n[1] * b.n[2];
  const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int nwave = gridDim.x * (kBlock / 64);
  for (int task = wave; task < ntask; task += nwave) {
    const int xc = task % nxc, rem = task / nxc, y = 1 + rem % b.n[1], z = 1 + rem / b.n[1];
    const int x0 = 1 + 16 * xc;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int xi = x0 + li;  // this lane's A row (point)
    const bool live = xi <= b.n[0];
    if (CIN == 16) {
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
        bf16x4 a = {0, 0, 0, 0};
        if (live) {
          const ushort4 v4 = *reinterpret_cast<const ushort4*>(in + (size_t)pg_pt(b, xi + dx, y + dy, z + dz) * 16 + 4 * lg);
          a[0] = (short)v4.x; a[1] = (short)v4.y; a[2] = (short)v4.z; a[3] = (short)v4.w;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[t], acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        const int t = 4 * q + lg;
        bf16x4 a = {0, 0, 0, 0};
        if (live && t < 27) {
          const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
          const ushort4 v4 = *reinterpret_cast<const ushort4*>(in + (size_t)pg_pt(b, xi + dx, y + dy, z + dz) * 4);
          a[0] = (short)v4.x; a[1] = (short)v4.y; a[2] = (short)v4.z; a[3] = (short)v4.w;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[q], acc, 0, 0, 0);
      }
    }
    // D[i = 4 lg + v][j = li]: point x0 + 4 lg + v, output channel li
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int xo = x0 + 4 * lg + v;
      if (xo > b.n[0]) continue;
      const size_t p = (size_t)pg_pt(b, xo, y, z);
      if (MODE == 0) {
        out[p * 16 + li] = f2bf(fmaxf(acc[v] + bj, 0.f));
      } else if (MODE == 1) {
        if (li == 0) outf[p] = acc[v] + bj;
      } else {
        const unsigned short r = ref[p * 16 + li];
        const bool pos = (r & 0x8000u) == 0 && r != 0;
        out[p * 16 + li] = pos ? f2bf(acc[v]) : (unsigned short)0;
      }
    }
  }
}

// Weight gradients of one layer: dW[t][ci][co] = sum_p in[p + off(t)][ci] g[p][co],
// db[co] = sum_p g[p][co], over the box interior.  MFMA with D[i = ci][j = co] and the
// points as K.  Each wave writes its partial (27*256 + 16 floats) to part[wave].
template <int CIN>
__global__ void __launch_bounds__(kBlock) k_pg_wgrad(PgBox b, const unsigned short* in,
                                                     const unsigned short* g, float* part) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float accb = 0.f;
  const int nxc = (b.n[0] + 15) / 16;
  const int ntask = nxc * b.n[1] * b.n[2];
  const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int nwave = gridDim.x * (kBlock / 64);
  for (int task = wave; task < ntask; task += nwave) {
    const int xc = task % nxc, rem = task / nxc, y = 1 + rem % b.n[1], z = 1 + rem / b.n[1];
    const int x0 = 1 + 16 * xc;
    // B[k = point 4 lg + v][j = co li] = g[point][co]
    bf16x4 bg;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int xp = x0 + 4 * lg + v;
      const unsigned short h = (xp <= b.n[0]) ? g[(size_t)pg_pt(b, xp, y, z) * 16 + li] : (unsigned short)0;
      bg[v] = (short)h;
      accb += bf2f(h);
    }
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
      // A[i = ci li][k = point 4 lg + v] = in[point + off(t)][ci]
      bf16x4 a;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int xp = x0 + 4 * lg + v;
        unsigned short h = 0;
        if (xp <= b.n[0] && li < CIN) h = in[(size_t)pg_pt(b, xp + dx, y + dy, z + dz) * CIN + li];
        a[v] = (short)h;
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bg, acc[t], 0, 0, 0);
    }
  }
  float* dst = part + (size_t)wave * (27 * 256 + 16);
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[t * 256 + (4 * lg + v) * 16 + li] = acc[t][v];
  // bias: lanes li, li+16, li+32, li+48 hold disjoint points of channel li
  accb += __shfl_down(accb, 32, 64);
  accb += __shfl_down(accb, 16, 64);
  if (lg == 0) dst[27 * 256 + li] = accb;
}

// Sum the per-wave partials into the flat FP32 gradient of one layer.
// cin_real / cout_real select the stored entries; grad_w, grad_b point into the flat vector.
__global__ void __launch_bounds__(kBlock) k_pg_wgrad_reduce(const float* part, int nparts, int cin_real,
                                                           int cout_real, float* grad_w, float* grad_b) {
  const int nw = 27 * cin_real * cout_real;
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nw + cout_real; e += gridDim.x * kBlock) {
    int src;
    if (e < nw) {
      const int co = e % cout_real, ci = (e / cout_real) % cin_real, t = e / (cout_real * cin_real);
      src = t * 256 + ci * 16 + co;
    } else {
      src = 27 * 256 + (e - nw);
    }
    float s = 0.f;
    for (int k = 0; k < nparts; ++k) s += part[(size_t)k * (27 * 256 + 16) + src];
    if (e < nw) grad_w[e] = s;
    else grad_b[e - nw] = s;
  }
}

// Adam on the FP32 master weights, then refresh the bfloat16 kernel weights:
// forward W1f[27][4][16], W2f[27][16][16], W3f[27][16][16] (co 0 real) and the
// backward-data weights W3b[27][16][16] (input channel 0 real), W2b[27][16][16]
// (taps mirrored, channel roles swapped).
struct PgWeights {
  unsigned short *w1f, *w2f, *w3f, *w3b, *w2b;
  float *b1, *b2, *b3;
};

__global__ void __launch_bounds__(kBlock) k_pg_adam(float* w, float* m, float* v, const float* g, float lr,
                                                   float b1, float b2, float c1, float c2, float eps, int update) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < kPgParams; e += gridDim.x * kBlock) {
    if (!update) continue;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

__global__ void __launch_bounds__(kBlock) k_pg_pack(const float* w, PgWeights k) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < 27 * 256; e += gridDim.x * kBlock) {
    const int t = e / 256, r = (e / 16) % 16, c = e % 16;  // [t][r][c]
    // forward layer 1: [t][ci<4][co], ci = 3 is padding
    if (r < 4) k.w1f[t * 64 + r * 16 + c] = (r < 3) ? f2bf(w[kPgW1 + (t * 3 + r) * 16 + c]) : (unsigned short)0;
    k.w2f[e] = f2bf(w[kPgW2 + (t * 16 + r) * 16 + c]);
    k.w3f[e] = (c == 0) ? f2bf(w[kPgW3 + t * 16 + r]) : (unsigned short)0;
    const int tm = 26 - t;  // mirrored tap
    // backward data of layer 3: in-channel r = 0 (dy), out-channel c = layer-3 input channel
    k.w3b[e] = (r == 0) ? f2bf(w[kPgW3 + tm * 16 + c]) : (unsigned short)0;
    // backward data of layer 2: in-channel r = layer-2 output co, out-channel c = layer-2 input ci
    k.w2b[e] = f2bf(w[kPgW2 + (tm * 16 + c) * 16 + r]);
  }
  const int tid = blockIdx.x * kBlock + threadIdx.x;
  if (tid < 16) {
    k.b1[tid] = w[kPgB1 + tid];
    k.b2[tid] = w[kPgB2 + tid];
  }
  if (tid == 0) k.b3[0] = w[kPgB3];
}

// Gradient of the mean-removed MSE: pass 1 sums e = y - t over the loss mask.
__global__ void __launch_bounds__(kBlock) k_pg_err(PgBox b, const float* y, const float* tgt,
                                                  const unsigned char* mask, double* part) {
  const int total = b.n[0] * b.n[1] * b.n[2];
  double s = 0.0, c = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int x = 1 + lin % b.n[0], yy = 1 + (lin / b.n[0]) % b.n[1], z = 1 + lin / (b.n[0] * b.n[1]);
    const int p = pg_pt(b, x, yy, z);
    if (mask[p]) {
      s += double(y[p] - tgt[p]);
      c += 1.0;
    }
  }
  s = block_sum(s);
  c = block_sum(c);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s;
    part[2 * blockIdx.x + 1] = c;
  }
}

// pass 2: g3[p][0] = bf16(2 (e - mean e)/n) on the mask, 0 elsewhere; loss partials.
__global__ void __launch_bounds__(kBlock) k_pg_dy(PgBox b, const float* y, const float* tgt,
                                                 const unsigned char* mask, const double* part, int nparts,
                                                 unsigned short* g3, double* lpart) {
  double s = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
    s += part[2 * i];
    c += part[2 * i + 1];
  }
  s = block_sum(s);
  c = block_sum(c);
  const double mean = c > 0 ? s / c : 0.0, n = c > 0 ? c : 1.0;
  const int total = b.n[0] * b.n[1] * b.n[2];
  double l = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    const int x = 1 + lin % b.n[0], yy = 1 + (lin / b.n[0]) % b.n[1], z = 1 + lin / (b.n[0] * b.n[1]);
    const int p = pg_pt(b, x, yy, z);
    float gv = 0.f;
    if (mask[p]) {
      const double d = double(y[p] - tgt[p]) - mean;
      l += d * d;
      gv = float(2.0 * d / n);
    }
    g3[(size_t)p * 16] = f2bf(gv);
  }
  l = block_sum(l);
  if (threadIdx.x == 0) lpart[blockIdx.x] = l / n;
}

// Inputs of the net on the solver grid: p1 = p_{m-1}, p2 = p_{m-2}, z = div u,
// normalised by mu and s (moments of p1 over active cells), written as
// channels-last bfloat16 on the box whose halo is the solver's ghost layer.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_pg_moments(Grid3 g, const T* p1, const T* iD, double* part) {
  const int total = g.n[0] * g.n[1] * g.n[2];
  double s = 0.0, s2 = 0.0, c = 0.0;
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    if (iD[idx] != T(0)) {
      const double v = double(p1[idx]);
      s += v;
      s2 += v * v;
      c += 1.0;
    }
  }
  s = block_sum(s);
  s2 = block_sum(s2);
  c = block_sum(c);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s;
    part[3 * blockIdx.x + 1] = s2;
    part[3 * blockIdx.x + 2] = c;
  }
}

// mu, s from the moments (single block); s = 1 if the spread vanishes
__global__ void __launch_bounds__(kBlock) k_pg_norm(const double* part, int nparts, double* scal) {
  double s = 0.0, s2 = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
    s += part[3 * i];
    s2 += part[3 * i + 1];
    c += part[3 * i + 2];
  }
  s = block_sum(s);
  s2 = block_sum(s2);
  c = block_sum(c);
  if (threadIdx.x == 0) {
    const double mu = c > 0 ? s / c : 0.0;
    double var = c > 0 ? s2 / c - mu * mu : 0.0;
    if (var < 0) var = 0;
    double sd = sqrt(var);
    if (!(sd > 0.0)) sd = 1.0;
    scal[0] = mu;
    scal[1] = sd;
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_pg_features(Grid3 g, PgBox b, Vec3<T> u, const T* p1, const T* p2,
                                                        const T* iD, const double* scal, double wdt,
                                                        unsigned short* X) {
  const double mu = scal[0], s = scal[1];
  const int total = g.n[0] * g.n[1] * g.n[2];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    ushort4 o = {0, 0, 0, 0};
    if (iD[idx] != T(0)) {
      T z = T(0);
      for (int a = 0; a < D; ++a) {
        const int op = (g.per[a] && I[a] == g.n[a]) ? -(g.n[a] - 1) * g.s[a] : g.s[a];
        z = z + (u.c[a][idx + op] - u.c[a][idx]);
      }
      o.x = f2bf(float((double(p1[idx]) - mu) / s));
      o.y = f2bf(float((double(p2[idx]) - mu) / s));
      o.z = f2bf(float(double(z) / (wdt * s)));
    }
    *reinterpret_cast<ushort4*>(X + (size_t)pg_pt(b, I[0], I[1], I[2]) * 4) = o;
  }
}

// Initial guess x0 = (p1 + s y) wdt on active cells, p1 wdt elsewhere.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_pg_guess(Grid3 g, PgBox b, const T* p1, const T* iD, const float* y,
                                                     const double* scal, double wdt, T* x) {
  const double s = scal[1];
  const int total = g.n[0] * g.n[1] * g.n[2];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < total; lin += gridDim.x * kBlock) {
    int I[3], idx;
    cell_of<D>(g, lin, I, idx);
    double pg = double(p1[idx]);
    if (iD[idx] != T(0)) pg += s * double(y[pg_pt(b, I[0], I[1], I[2])]);
    x[idx] = T(pg * wdt);
  }
}

// Training snapshot: copy a kPgCrop^3 crop (origin o, interior coordinates) of the
// features, the target d* = (x/wdt - p1)/s and the active mask into a ring slot.
// The crop box has a zero halo; the loss mask excludes 3 cells at every crop face
// (the receptive field of the net stays inside the crop).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_pg_crop(Grid3 g, PgBox bd, const unsigned short* X, const T* x,
                                                    const T* p1, const T* iD, const double* scal, double wdt,
                                                    int ox, int oy, int oz, PgBox bc, unsigned short* Xc,
                                                    float* tc, unsigned char* mc) {
  const double s = scal[1];
  const int C0 = bc.n[0], C1 = bc.n[1], C2 = bc.n[2];
  for (int lin = blockIdx.x * kBlock + threadIdx.x; lin < C0 * C1 * C2; lin += gridDim.x * kBlock) {
    const int cx = 1 + lin % C0, cy = 1 + (lin / C0) % C1, cz = 1 + lin / (C0 * C1);
    const int I0 = ox + cx - 1, I1 = oy + cy - 1, I2 = oz + cz - 1;
    const int idx = I0 + I1 * g.s[1] + I2 * g.s[2];
    const int pc = pg_pt(bc, cx, cy, cz);
    *reinterpret_cast<ushort4*>(Xc + (size_t)pc * 4) =
        *reinterpret_cast<const ushort4*>(X + (size_t)pg_pt(bd, I0, I1, I2) * 4);
    const bool act = iD[idx] != T(0);
    tc[pc] = act ? float((double(x[idx]) / wdt - double(p1[idx])) / s) : 0.f;
    const bool inner = cx > 3 && cx <= C0 - 3 && cy > 3 && cy <= C1 - 3 && cz > 3 && cz <= C2 - 3;
    mc[pc] = (act && inner) ? 1 : 0;
  }
}

}  // namespace wl

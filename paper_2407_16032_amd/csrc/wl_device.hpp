// Device-side helpers shared by the BDIM step kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wl {

constexpr int kBlock = 256;       // threads per block (4 waves of 64)
constexpr int kMaxBlocks = 8192;  // no launch that writes partial sums exceeds this
constexpr int kGridStride = 2048; // grid-stride launches use at most this many blocks
constexpr int kFrontPad = 15;     // elements before every field, so interior rows start 64-B aligned
constexpr int kMaxLevels = 16;
constexpr int kMaxPcg = 15;

// reduction slots (each kMaxBlocks doubles)
constexpr int kSlotRho0 = 0;                   // rho_k for k = 0..kMaxPcg
constexpr int kSlotSig0 = kMaxPcg + 1;         // sigma_k for k = 0..kMaxPcg-1
constexpr int kSlotRmax = 2 * kMaxPcg + 1;     // residual max-norm
constexpr int kSlotCfl = kSlotRmax + 1;        // max outflux
constexpr int kSlotExit = kSlotCfl + 1;        // exit-plane flux
constexpr int kSlotForce = kSlotExit + 1;      // 11 slots: sum p n K (3), viscous (3), sum n K (3),
                                               // sum p and count over active cells
constexpr int kSlotSumR = kSlotForce + 11;     // sum of the residual over active cells
constexpr int kSlotCnt = kSlotSumR + 1;        // number of active cells
constexpr int kSlotL2 = kSlotCnt + 1;          // sum of the squared residual
constexpr int kSlotDiv = kSlotL2 + 1;          // max |div u| over active cells
constexpr int kNumSlots = kSlotDiv + 1;

// scalar results (doubles)
constexpr int kScalRmax = 0;
constexpr int kScalCfl = 1;
constexpr int kScalExitShift = 2;
constexpr int kScalL2 = 3;   // squared residual 2-norms of the predictor (3) and corrector (4) solves
constexpr int kScalDiv = 5;  // max |div u| after the step
constexpr int kNumScal = 8;

// One grid level.  n[2] = 1 and s[2] unused in 2-D.
struct Grid3 {
  int n[3];    // interior cells
  int s[3];    // element strides, s[0] = 1
  int per[3];  // periodic flags
};

template <typename T>
struct Vec3 {
  T* c[3];
};
template <typename T>
struct Vec9 {
  T* c[9];
};

// Periodic wrap of a padded coordinate x in [-1, N+2] into 1..N (no-op otherwise).
__device__ __forceinline__ int wrapc(int x, int a, const Grid3& g) {
  if (g.per[a]) {
    const int N = g.n[a];
    if (x < 1) x += N;
    else if (x > N) x -= N;
  }
  return x;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Block-wide reductions over NT threads (1-D block); every thread receives the
// result.  Fixed order: wave tree, then the waves in order, so results are
// bitwise reproducible run to run.
template <int NT = kBlock>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[NT / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}
template <int NT = kBlock>
__device__ __forceinline__ double block_max(double v) {
  __shared__ double shm[NT / 64];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) shm[w] = v;
  __syncthreads();
  double r = shm[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) r = fmax(r, shm[i]);
  __syncthreads();
  return r;
}

// Sum / max of the n per-block partials a producer kernel wrote.
template <int NT = kBlock>
__device__ __forceinline__ double total_of(const double* part, int n) {
  if (n == 1) return part[0];  // already reduced (uniform over the grid)
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) v += part[i];
  return block_sum<NT>(v);
}
template <int NT = kBlock>
__device__ __forceinline__ double max_of(const double* part, int n) {
  if (n == 1) return part[0];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) v = fmax(v, part[i]);
  return block_max<NT>(v);
}

// Number of partials each consumed slot holds (the producer's grid size).
struct RedN {
  int mean;      // kSlotSumR / kSlotCnt
  int rho;       // rho_k
  int rho_prev;  // rho_{k-1}
  int sig;       // sigma_k
};

// 16-byte vector of T for the flat (pointwise) kernels
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; static constexpr int W = 4; };
template <> struct Vec16<double> { typedef double2 type; static constexpr int W = 2; };

// Streaming stores and loads: fields of the large levels are several times the
// size of the last-level cache and are touched once per pass, so their stores
// (and the loads no neighbouring tile re-reads) carry the non-temporal hint.
#ifndef WL_NT_MODE
#define WL_NT_MODE 1
#endif
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
#if WL_NT_MODE >= 1
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
#if WL_NT_MODE >= 2
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

template <typename T>
__device__ __forceinline__ T median3(T a, T b, T c) {
  return fmax(fmin(a, b), fmin(fmax(a, b), c));
}
// the same median in one instruction (finite arguments; the result is one of them)
template <>
__device__ __forceinline__ float median3<float>(float a, float b, float c) {
  return __builtin_amdgcn_fmed3f(a, b, c);
}

// kappa = 1/3 upwind-biased face value, clamped by the median-form limiter.
template <typename T>
__device__ __forceinline__ T quick_lim(T far, T c, T d) {
  const T q = (T(5) * c + T(2) * d - far) * T(1.0 / 6.0);  // a product: the divide is a long sequence
  return median3(c, q, median3(c, d, c + T(9) * (c - far)));
}

}  // namespace wl

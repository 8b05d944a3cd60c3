// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define P3MZ_MAX_CYCLES 64
#define P3MZ_MAX_LEVELS 16
#define P3MZ_MAX_ORDER 7
#define P3MZ_TAIL_MAX 16        // levels of at most 16^3 run in one LDS-resident workgroup
#define P3MZ_TAIL_MAX_BATCH 32  // batched systems: the 32^3 level joins that workgroup (in global memory)
#define P3MZ_WAVE 64

// Device-side control block.  Kernels of the V-cycle read `done` first and
// return at once when the solve has converged, so a fixed launch sequence
// (or a replayed graph) can hold more cycles than a step needs.  The cycle
// index and the rotation of the potential/multiplier history also live here,
// so captured graphs never need new kernel arguments.
struct Ctl {
  // solve state of the current step (read back by the host after the solve)
  int done;              // 1: converged or cycle cap reached
  int cycles;            // V-cycles applied this step
  int status;            // 0 ok, 1 cycle cap reached
  int final_buf;         // which y ping-pong buffer holds the final multiplier
  int nan_flag;          // non-finite position seen by a binning kernel
  // history: advanced on the device at the end of every step
  int cold;              // this step starts from a zero potential
  int m_eff;             // predictor order of this step
  int n_yh;              // stored warm multipliers (0..3)
  int k_idx;             // phi buffer holding phi^k
  int yh0, yh1, yh2;     // multiplier buffers, newest first
  int predictor;         // requested predictor order
  int md_step;           // row of the MD energy log
  int pending;           // 1 + cycle of an outer residual whose stop decision is still to be made (0: none)
  int nbr_stale;         // 1: the short-range neighbour list must be rebuilt this step
  long long steps;       // completed steps
  double thresh;         // residual threshold
  double norm_qs;        // max |q^s|
  double mean_sigma;     // mean of the unprojected sigma_p
  double mean_y;         // mean of the current multiplier
  double e_lr, e_sr;
  double res_hist[P3MZ_MAX_CYCLES + 1];
  long long nbr_builds;  // neighbour-list builds so far
  int nbr_over;          // atoms whose neighbours exceeded the list capacity at the last build
  int pad2;
  long long therm_step;  // MD steps since the thermostat was set (counter of its random numbers)
  double net_force[3];   // sum of the step's electrostatic forces (NaN when no force was written)
};

// Langevin thermostat of the OVRVO splitting: v <- a v + b sqrt(kT / (m e)) z
// at both ends of a step (e = the mass-velocity-to-energy factor), z standard
// normals from the counter-based generator keyed by seed.
struct Thermostat {
  int on;
  double a, b, kt, mv2e;
  unsigned seed0, seed1;
  const Ctl* ctl;   // therm_step
};

// --- wave / block reductions (wave64) ------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum / max with a fixed reduction tree (deterministic for a fixed
// block size).  `sh` needs blockDim.x/64 doubles.  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; i++) r += sh[i];
  return r;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; i++) r = fmax(r, sh[i]);
  return r;
}

// Max and sum of one value per thread in one pass (one pair of barriers);
// `sh` needs 2 * blockDim.x/64 doubles.  Results valid in thread 0.
__device__ __forceinline__ void block_max_sum(double* mx, double* sm, double* sh) {
  const double m = wave_max(*mx), v = wave_sum(*sm);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) {
    sh[w] = m;
    sh[nw + w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nw; i++) {
      a = fmax(a, sh[i]);
      b += sh[nw + i];
    }
    *mx = a;
    *sm = b;
  }
}

// Reductions are two-pass: every workgroup of a kernel stores its partial,
// then a one-workgroup kernel reads them in index order (kernel boundaries
// make the partials visible across XCDs without device-scope fences in the
// hot kernels).  Deterministic sum of n partials: fixed strided split + fixed tree.
__device__ __forceinline__ double reduce_partials_sum(const double* p, int n, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += p[i];
  return block_sum(acc, sh);
}
__device__ __forceinline__ double reduce_partials_max(const double* p, int n, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc = fmax(acc, p[i]);
  return block_max(acc, sh);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Renumbering them so that each XCD walks one contiguous eighth
// of the index space keeps stencil neighbours (adjacent rows and planes) in
// the same XCD's L2 instead of re-reading them from HBM on another XCD.
__device__ __forceinline__ int xcd_block() {
  const int g = gridDim.x, b = blockIdx.x;
  if (g & 7) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// Reduction kernels use a capped grid: each (XCD-renumbered) workgroup walks
// one contiguous chunk of the index space, a multiple of the block size.
constexpr int kRedBlock = 256;
constexpr int kMaxRedBlocks = 2048;
// Capacity (doubles) of a context's partial-sum buffer.  Every reduction
// launch writes at most this many partials: two per workgroup on grids of
// at most kMaxRedBlocks (sigma, outer residual), one per workgroup on grids
// of at most kPartialSlots (pair kernels, wave per atom) or kMaxRedBlocks
// (gather, kinetic energy).
constexpr int kPartialSlots = 2 * kMaxRedBlocks;
inline int red_blocks(int64_t count) {
  int64_t b = (count + kRedBlock - 1) / kRedBlock;
  if (b > kMaxRedBlocks) b = kMaxRedBlocks;
  if (b >= 8) b &= ~7LL;
  return (int)(b < 1 ? 1 : b);
}
__device__ __forceinline__ void chunk_range(int64_t count, int* lo, int* hi) {
  const int64_t g = gridDim.x;
  int64_t per = (count + g - 1) / g;
  per = (per + kRedBlock - 1) / kRedBlock * kRedBlock;
  const int64_t l = (int64_t)xcd_block() * per;
  *lo = (int)(l < count ? l : count);
  *hi = (int)(l + per < count ? l + per : count);
}

// Piecewise Chebyshev table of erfcx(x) = exp(x^2) erfc(x) on [0, X]:
// intervals of width X/n, degree kErfcDeg; coefficient j of interval k at
// [k * (kErfcDeg + 1) + j], the constant term already halved.
constexpr int kErfcDeg = 11;
constexpr int kErfcMaxIntervals = 128;

// erfcx(x) for 0 <= x < n / scale, from a table in LDS (Clenshaw).
__device__ __forceinline__ double erfcx_table(const double* tab, int n, double scale, double x) {
  const double u = x * scale;
  int k = (int)u;
  k = k < n - 1 ? k : n - 1;
  const double t = 2.0 * (u - (double)k) - 1.0;
  const double* c = tab + k * (kErfcDeg + 1);
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int j = kErfcDeg; j >= 1; j--) {
    const double b0 = fma(2.0 * t, b1, c[j] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(t, b1, c[0] - b2);
}

// --- mesh indexing ---------------------------------------------------------
// Natural layout: x fastest.  Colour-split layout: the points of colour
// c = (i+j+k)&1 of each row (j,k) are packed, index ((k*n + j)*(n/2) + i/2).
__device__ __forceinline__ int nat_idx(int n, int i, int j, int k) { return (k * n + j) * n + i; }
__device__ __forceinline__ int cs_idx(int n, int i, int j, int k) { return (k * n + j) * (n >> 1) + (i >> 1); }
__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// B-spline weights of order p at fractional offset tau in [0,1):
// w[j] = M_p(tau + p - 1 - j), built by the triangular de Boor recursion
// w_j^(k) = ((tau + k-1-j) w_{j-1}^(k-1) + (1 - tau + j) w_j^(k-1)) / (k-1).
template <typename T>
__device__ __forceinline__ void bspline_weights(int p, T tau, T* w) {
  w[0] = T(1);
  for (int k = 2; k <= p; k++) {
    T inv = T(1) / T(k - 1);
    T prev = T(0);   // w_{j-1}^{(k-1)}
    for (int j = 0; j < k; j++) {
      T cur = (j < k - 1) ? w[j] : T(0);
      w[j] = ((tau + T(k - 1 - j)) * prev + (T(1) - tau + T(j)) * cur) * inv;
      prev = cur;
    }
  }
}

// Host-side error helper.
#define P3MZ_HIP_TRY(expr)                        \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __FILE__, __LINE__); \
  } while (0)

// Mesh-side kernels of the step: charge smoothing, constraint at the Verlet
// prediction, outer FP64 residual, the multigrid V-cycle on colour-split
// (red/black) storage, and the field update.
#include "kern.h"
#include "launch.h"

namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

// Geometry of one power-of-two level in colour-split layout (see the V-cycle
// kernels below); all index arithmetic is shifts and masks.
struct CsGeo {
  int l2, n, hn, plane;   // edge n = 2^l2, half edge, elements per z-plane of one colour
  __device__ explicit CsGeo(int n_) : l2(__builtin_ctz(n_)), n(n_), hn(n_ >> 1), plane(n_ * (n_ >> 1)) {}
};

__device__ __forceinline__ void cs_decode(const CsGeo& g, int t, int* m, int* j, int* k) {
  *m = t & (g.hn - 1);
  const int row = t >> (g.l2 - 1);
  *j = row & (g.n - 1);
  *k = row >> g.l2;
}

__device__ __forceinline__ int cs_index(const CsGeo& g, int i, int j, int k) {
  return (((k << g.l2) + j) << (g.l2 - 1)) + (i >> 1);
}


// ---------------------------------------------------------------------------
// Smoothing: one periodic line filter along `AXIS` (0 = x, 1 = y, 2 = z).
// The K-fold diffusion step [nu, 1-2nu, nu] is applied as its (2K+1)-tap
// convolution, folded onto the periodic line when 2K+1 > n:
// out[i] = sum_m taps[m] v[(i + m - half) mod n], m ascending.
// A workgroup owns W lines and a segment of S consecutive outputs of each
// (S divides n; whole lines when they fit in LDS).  It stages the segment
// extended by the filter reach, ext[k] = v[(i_seg + k - half) mod n] for
// k < S + kt + R, so no index wraps inside the filter loop; kt is ntaps
// rounded up to a multiple of R with zero taps (they add exact zeros).
// Each thread produces R consecutive outputs of one line: taps are taken R
// at a time with a window of 2R line values in registers, and every output
// sums its terms in ascending tap order.  y/z lines are W consecutive x
// columns (coalesced loads and stores), staged position-major; x lines are
// staged row-major and written back through a second LDS buffer so the
// global stores stay coalesced.
// ---------------------------------------------------------------------------
template <typename T, int AXIS, int W, int R>
struct Smooth {
  struct Args {
    int n, ntaps, half, seg;
    const T *taps, *in;
    T* out;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};

// LDS layout of one smoothing workgroup (elements): the padded taps, the
// staged extended lines and, for x lines, the output rows.
struct SmoothLds {
  int kt, L, ld, ldo, taps_off, buf_off, obuf_off, total;
  // vw: elements per 16 bytes (2 for FP64, 4 for FP32)
  __host__ __device__ SmoothLds(int axis, int W, int R, int ntaps, int seg, int vw = 2) {
    kt = (ntaps + R - 1) / R * R;
    L = seg + kt + R;
    ld = axis == 0 ? ((L + 15) & ~15) + vw : W + 1;   // 16-byte rows, staggered over the banks
    ldo = seg + 2;
    taps_off = 0;
    buf_off = (kt + vw - 1) / vw * vw;
    obuf_off = buf_off + (axis == 0 ? W * ld : L * ld);
    total = obuf_off + (axis == 0 ? W * ldo : 0);
  }
};

template <typename T, int AXIS, int W, int R>
__device__ void Smooth<T, AXIS, W, R>::run(const Args& A, Grid G) {
  static_assert((W & (W - 1)) == 0 && R % 2 == 0, "W a power of two, R even");
  const int n = A.n, ntaps = A.ntaps, half = A.half, S = A.seg, msk = n - 1;
  const T* __restrict__ in = A.in;
  T* __restrict__ out = A.out;
  const SmoothLds lay(AXIS, W, R, ntaps, S, 16 / (int)sizeof(T));
  extern __shared__ __align__(16) unsigned char smooth_lds[];
  T* const lds = reinterpret_cast<T*>(smooth_lds);
  T* const taps = lds + lay.taps_off;
  T* const buf = lds + lay.buf_off;
  const int kt = lay.kt, L = lay.L, ld = lay.ld;
  const int tid = threadIdx.x;
  for (int i = tid; i < kt; i += kBlock) taps[i] = i < ntaps ? A.taps[i] : T(0);
  // workgroup -> (line group, segment)
  const int nseg = n / S;
  const int seg = G.b % nseg, grp = G.b / nseg;
  const int i_seg = seg * S;
  size_t row0 = 0;
  int x0 = 0, o = 0;
  // Staging: the loads of a batch are all issued before the first LDS
  // store, so their memory round trips overlap (a load followed at once by
  // its store would wait for each in turn).
  if (AXIS == 0) {
    row0 = (size_t)grp * W;
    // one position k of all W lines per batch
    for (int kc = 0; kc < L; kc += kBlock) {
      const int k = kc + tid;
      const bool ok = k < L;
      const size_t src = (size_t)((i_seg + k - half) & msk);
      T v[W];
#pragma unroll
      for (int r = 0; r < W; r++) v[r] = ok ? in[(row0 + r) * n + src] : T(0);
      if (ok) {
#pragma unroll
        for (int r = 0; r < W; r++) buf[r * ld + k] = v[r];
      }
    }
  } else {
    const int ncol = n / W;
    x0 = (grp % ncol) * W;
    o = grp / ncol;
    constexpr int B = 8;   // elements per thread and batch
    for (int e0 = tid; e0 < L * W; e0 += B * kBlock) {
      T v[B];
#pragma unroll
      for (int u = 0; u < B; u++) {
        const int e = e0 + u * kBlock;
        const int k = e / W, c = e & (W - 1);
        const int t = (i_seg + k - half) & msk;
        const size_t a = AXIS == 1 ? ((size_t)o * n + t) * n + x0 + c : ((size_t)t * n + o) * n + x0 + c;
        v[u] = e < L * W ? in[a] : T(0);
      }
#pragma unroll
      for (int u = 0; u < B; u++) {
        const int e = e0 + u * kBlock;
        if (e < L * W) buf[(e / W) * ld + (e & (W - 1))] = v[u];
      }
    }
  }
  __syncthreads();
  T* const obuf = lds + lay.obuf_off;
  for (int task = tid; task < W * (S / R); task += kBlock) {
    const int c = task & (W - 1), i0 = (task / W) * R;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; r++) acc[r] = T(0);
    for (int m0 = 0; m0 < kt; m0 += R) {
      T v[2 * R], tp[R];
      if (AXIS == 0) {
        if constexpr (sizeof(T) == 8) {
          const double2* p = reinterpret_cast<const double2*>(buf + c * ld + i0 + m0);
#pragma unroll
          for (int q = 0; q < R; q++) {
            const double2 d = p[q];
            v[2 * q] = d.x;
            v[2 * q + 1] = d.y;
          }
        } else {
          const float4* p = reinterpret_cast<const float4*>(buf + c * ld + i0 + m0);
#pragma unroll
          for (int q = 0; q < R / 2; q++) {
            const float4 d = p[q];
            v[4 * q] = d.x;
            v[4 * q + 1] = d.y;
            v[4 * q + 2] = d.z;
            v[4 * q + 3] = d.w;
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < 2 * R; q++) v[q] = buf[(i0 + m0 + q) * ld + c];
      }
#pragma unroll
      for (int j = 0; j < R; j++) tp[j] = taps[m0 + j];
#pragma unroll
      for (int j = 0; j < R; j++)
#pragma unroll
        for (int r = 0; r < R; r++) acc[r] += tp[j] * v[r + j];
    }
    if (AXIS == 0) {
#pragma unroll
      for (int r = 0; r < R; r++) obuf[c * lay.ldo + i0 + r] = acc[r];
    } else {
#pragma unroll
      for (int r = 0; r < R; r++) {
        const int t = i_seg + i0 + r;
        const size_t a = AXIS == 1 ? ((size_t)o * n + t) * n + x0 + c : ((size_t)t * n + o) * n + x0 + c;
        out[a] = acc[r];
      }
    }
  }
  if (AXIS == 0) {
    __syncthreads();
    for (int r = 0; r < W; r++)
      for (int i = tid; i < S; i += kBlock) out[(row0 + r) * n + i_seg + i] = obuf[r * lay.ldo + i];
  }
}

// ---------------------------------------------------------------------------
// Constraint at the Verlet prediction (Eq. 17) and multiplier predictor.
// Reduction kernels run on a capped grid (each workgroup walks one contiguous
// chunk), so their one-workgroup finalize pass reads few partials.
// ---------------------------------------------------------------------------
// Four consecutive FP64 values of a natural-layout array (t a multiple of 4:
// 32-byte aligned, one row of the mesh).
struct D4 {
  double v[4];
};
__device__ __forceinline__ D4 ld4(const double* __restrict__ a, int t) {
  const double2 lo = *reinterpret_cast<const double2*>(a + t), hi = *reinterpret_cast<const double2*>(a + t + 2);
  return D4{{lo.x, lo.y, hi.x, hi.y}};
}
__device__ __forceinline__ void st4(double* __restrict__ a, int t, const double* v) {
  *reinterpret_cast<double2*>(a + t) = make_double2(v[0], v[1]);
  *reinterpret_cast<double2*>(a + t + 2) = make_double2(v[2], v[3]);
}

// Visits the n^3 points of a natural-layout mesh four at a time (x-vectors
// of one row), calling f(t) with the index of the first point.  From 64^3 up
// a workgroup walks a column: JB consecutive rows (the 1024 points of one
// pass of 256 threads) of a band of z-planes, plane after plane, so a 7-point
// stencil's z-neighbour rows are those the workgroup read one pass before or
// reads one pass later; the workgroups of one XCD (consecutive logical
// indices) cover every column of the same z-band, so y-neighbour rows are
// shared through that XCD's L2.  The grid is red_blocks(n^3 / 4), which for
// n >= 64 is (n / JB) columns times a whole number of z-bands.  Smaller
// meshes take contiguous chunks.
template <typename F>
__device__ __forceinline__ void march4(const Grid& G, int n, F f) {
  const int l2 = __builtin_ctz(n), msk = n - 1;
  if (n >= 64) {
    const int JB = (4 * kBlock) >> l2, nj = n / JB, nz = G.g / nj, KB = n / nz;
    const int jb = G.b % nj, zr = G.b / nj;
    const int j = jb * JB + ((4 * (int)threadIdx.x) >> l2), x = (4 * (int)threadIdx.x) & msk;
    for (int kk = 0; kk < KB; kk++) {
      const int k = zr * KB + kk;
      f(((k << l2) + j) * n + x);
    }
  } else {
    int lo, hi;
    chunk_range(G, n * n * n, &lo, &hi);
    for (int t = lo + 4 * threadIdx.x; t < hi; t += 4 * kBlock) f(t);
  }
}

// Column walk with the rows of a plane shared through LDS (meshes from
// 256^3 up, single systems).  A workgroup of NT threads owns JB = 4 NT / n
// consecutive rows (four points of one row per thread; a wave lies within one
// row) of a band of KB z-planes and walks it plane after plane.  The rows of
// planes k-1, k and k+1 at a thread's own points stay in registers; plane k's
// JB rows plus one halo row on each side sit in LDS, where the y-neighbour
// rows are read, and the x-neighbours at the ends of a thread's four points
// come from the neighbouring lanes (from LDS at the ends of a wave).  Every
// row, halo rows included, is loaded from memory once per workgroup, one
// plane ahead of its use; a halo row is the neighbouring column's own row of
// the same plane, loaded by it at about the same time.  The grid is
// (n / JB) columns times nz z-bands; the LDS is two plane buffers of
// (JB + 2) n doubles (dynamic, col_lds_bytes).  load(i0, j, k) returns the
// four values at (i0.., j, k); point(t, i0, j, k, own, ym, yp, zm, zp, xl, xr)
// consumes a plane's four points.  Every thread runs the same KB iterations,
// each ending in one workgroup barrier.
constexpr int kColThreads = 512;   // workgroup of the shared-row column walk
constexpr int kColPerCu = 2;       // its workgroups per compute unit
// Single systems (not recorded into a batch) from 256^3 up: a wave then lies
// within one row and 2 (4 NT / n + 2) n doubles fit in LDS.
inline bool col_walk_on(int n) { return n >= 256 && n <= 512 && !g_recorder; }
template <int NT>
__device__ __forceinline__ int col_rows(int n) { return (4 * NT) / n; }
inline size_t col_lds_bytes(int nt, int n) { return 2 * (size_t)(4 * nt + 2 * n) * sizeof(double); }
// Workgroups of the shared-row column walk: n / JB columns times z-bands,
// about `per_cu` workgroups per compute unit.
inline int col_grid(int nt, int n, int per_cu) {
  const int jb = 4 * nt / n, nj = n / jb;
  int nz = 1;
  while (nz < n && nj * nz < 256 * per_cu) nz *= 2;
  return nj * nz;
}

template <int NT, typename LoadF, typename PointF>
__device__ __forceinline__ void col_walk(const Grid& G, int n, double* lds, LoadF load, PointF point) {
  const int l2 = __builtin_ctz(n), msk = n - 1;
  const int JB = col_rows<NT>(n), nj = n / JB, nz = G.g / nj, KB = n / nz;
  const int jb = G.b % nj, zr = G.b / nj;
  const int tid = threadIdx.x, lane = tid & 63;
  const int jl = (4 * tid) >> l2, i0 = (4 * tid) & msk;
  const int j0 = jb * JB, j = j0 + jl, k0 = zr * KB;
  const int row_len = n;   // doubles per LDS row
  const int buf_len = (JB + 2) * n;
  // halo rows: threads [0, n/4) hold row j0 - 1 (LDS row 0), threads
  // [n/4, n/2) row j0 + JB (LDS row JB + 1)
  const bool halo = tid < (n >> 1);
  const bool lower = tid < (n >> 2);
  const int hrow = lower ? 0 : JB + 1;
  const int hj = (lower ? j0 - 1 : j0 + JB) & msk;
  auto put = [&](double* b, int row, int x, const D4& v) {
    double2* p = reinterpret_cast<double2*>(b + row * row_len + x);
    p[0] = make_double2(v.v[0], v.v[1]);
    p[1] = make_double2(v.v[2], v.v[3]);
  };
  auto get = [&](const double* b, int row, int x) {
    const double2* p = reinterpret_cast<const double2*>(b + row * row_len + x);
    const double2 lo = p[0], hi = p[1];
    return D4{{lo.x, lo.y, hi.x, hi.y}};
  };
  double* cur = lds;
  double* nxt = lds + buf_len;
  D4 zm = load(i0, j, (k0 - 1) & msk);
  D4 own = load(i0, j, k0);
  put(cur, jl + 1, i0, own);
  if (halo) put(cur, hrow, i0, load(i0, hj, k0));
  __syncthreads();
  for (int kk = 0; kk < KB; kk++) {
    const int k = k0 + kk, kp = (k + 1) & msk;
    const D4 zp = load(i0, j, kp);
    D4 hz{{0.0, 0.0, 0.0, 0.0}};
    if (halo) hz = load(i0, hj, kp);
    const D4 ym = get(cur, jl, i0), yp = get(cur, jl + 2, i0);
    double xl = __shfl_up(own.v[3], 1, 64), xr = __shfl_down(own.v[0], 1, 64);
    if (lane == 0) xl = cur[(jl + 1) * row_len + ((i0 - 1) & msk)];
    if (lane == 63) xr = cur[(jl + 1) * row_len + ((i0 + 4) & msk)];
    point(((k << l2) + j) * n + i0, i0, j, k, own, ym, yp, zm, zp, xl, xr);
    put(nxt, jl + 1, i0, zp);
    if (halo) put(nxt, hrow, i0, hz);
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
    zm = own;
    own = zp;
  }
}

// Partials of a reduction kernel at stride nbp (the count its consumers
// read): this launch's G.g slots, and zeros (neutral for the max and the sum)
// in the rest when its grid is smaller.
__device__ __forceinline__ void put_partials(double* partial, int nbp, const Grid& G, double a, double b) {
  if (threadIdx.x == 0) {
    partial[G.b] = a;
    partial[nbp + G.b] = b;
  }
  for (int s = G.g + G.b * (int)blockDim.x + (int)threadIdx.x; s < nbp; s += G.g * (int)blockDim.x) {
    partial[s] = 0.0;
    partial[nbp + s] = 0.0;
  }
}

template <typename TQ>
struct SigmaArgs {
  int n;
  double h;
  const TQ* qs;
  const double *phi0, *phi1, *yb0, *yb1, *yb2;
  double *sigma, *y, *partial;
  const Ctl* ctl;
  int nbp;   // partial stride (>= the grid)
};
// NT > kBlock: the shared-row column walk (n >= 256)
template <typename TQ, int NT = kBlock>
struct Sigma {
  using Args = SigmaArgs<TQ>;
  static constexpr int kThreads = NT;
  __device__ static void run(const Args& A, Grid G);
};
// Four consecutive values of the smoothed charges, widened to FP64.
__device__ __forceinline__ D4 ld4q(const double* __restrict__ a, int t) { return ld4(a, t); }
__device__ __forceinline__ D4 ld4q(const float* __restrict__ a, int t) {
  const float4 v = *reinterpret_cast<const float4*>(a + t);
  return D4{{(double)v.x, (double)v.y, (double)v.z, (double)v.w}};
}

template <typename TQ, int NT>
__device__ void Sigma<TQ, NT>::run(const Args& A, Grid G) {
  const int n = A.n;
  const double h = A.h;
  const TQ* __restrict__ qs = A.qs;
  const double* __restrict__ phi0 = A.phi0;
  const double* __restrict__ phi1 = A.phi1;
  const double* __restrict__ yb0 = A.yb0;
  const double* __restrict__ yb1 = A.yb1;
  const double* __restrict__ yb2 = A.yb2;
  double* __restrict__ sigma = A.sigma;
  double* __restrict__ y = A.y;
  double* __restrict__ partial = A.partial;
  const Ctl* ctl = A.ctl;
  __shared__ double sh[NT / 64];
  const int cold = ctl->cold, m_eff = ctl->m_eff;
  const double* pk = ctl->k_idx ? phi1 : phi0;
  const double* pkm1 = ctl->k_idx ? phi0 : phi1;
  const double* const yb[3] = {yb0, yb1, yb2};
  const double* y0 = yb[ctl->yh0];
  const double* y1 = yb[ctl->yh1];
  const double* y2 = yb[ctl->yh2];
  double sv = 0.0, qmax = 0.0;
  const int l2 = __builtin_ctz(n), msk = n - 1;
  // Verlet-predicted potential P = 2 phi^k - phi^{k-1} on four points of a row
  auto P4 = [&](int a) {
    const D4 u = ld4(pk, a), w = ld4(pkm1, a);
    D4 r;
#pragma unroll
    for (int c = 0; c < 4; c++) r.v[c] = 2.0 * u.v[c] - w.v[c];
    return r;
  };
  auto P1 = [&](int a) { return 2.0 * pk[a] - pkm1[a]; };
  // sigma_p and the predicted y of four points from the P rows of the
  // point and its y and z neighbours and the x-neighbours xl, xr of its
  // first and last point (unused on a cold solve)
  auto point4 = [&](int t, int i0, int j, int k, const D4& own, const D4& ym, const D4& yp, const D4& zm,
                    const D4& zp, double xl, double xr) {
    const D4 q4 = ld4q(qs, t);
    double sg[4];
#pragma unroll
    for (int c = 0; c < 4; c++) sg[c] = q4.v[c];
    if (!cold) {
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const double xm = c == 0 ? xl : own.v[c - 1], xp = c == 3 ? xr : own.v[c + 1];
        const double nb = ((xm + xp) + (ym.v[c] + yp.v[c])) + (zm.v[c] + zp.v[c]);
        const double mphi = nb - 6.0 * own.v[c];
        sg[c] = h / (4.0 * kPi) * mphi + q4.v[c];
      }
    }
    st4(sigma, t, sg);
    double yv[4] = {0.0, 0.0, 0.0, 0.0};
    if (m_eff >= 1) {
      const D4 a0 = ld4(y0, t);
      D4 a1 = a0, a2 = a0;
      if (m_eff >= 2) a1 = ld4(y1, t);
      if (m_eff >= 3) a2 = ld4(y2, t);
#pragma unroll
      for (int c = 0; c < 4; c++) {
        if (m_eff == 1) yv[c] = a0.v[c];
        else if (m_eff == 2) yv[c] = 2.0 * a0.v[c] - a1.v[c];
        else yv[c] = 3.0 * a0.v[c] - 3.0 * a1.v[c] + a2.v[c];
      }
    }
    st4(y, t, yv);
#pragma unroll
    for (int c = 0; c < 4; c++) {
      sv += sg[c];
      qmax = fmax(qmax, fabs(q4.v[c]));
    }
  };
  const D4 zero4{{0.0, 0.0, 0.0, 0.0}};
  // x-neighbours of the four points at t (row start t - i0)
  auto xlr = [&](int t, int i0, double* xl, double* xr) {
    *xl = *xr = 0.0;
    if (!cold) {
      *xl = P1(t - i0 + ((i0 - 1) & msk));
      *xr = P1(t - i0 + ((i0 + 4) & msk));
    }
  };
  if constexpr (NT > kBlock) {
    extern __shared__ __align__(16) double col_lds[];
    col_walk<NT>(G, n, col_lds, [&](int i0, int j, int k) { return cold ? zero4 : P4(nat_idx(n, i0, j, k)); },
                 [&](int t, int i0, int j, int k, const D4& own, const D4& ym, const D4& yp, const D4& zm,
                     const D4& zp, double xl, double xr) { point4(t, i0, j, k, own, ym, yp, zm, zp, xl, xr); });
  } else if (n >= 64) {
    // the column walk of march4 with the z-neighbour rows of P kept in
    // registers from plane to plane
    const int JB = (4 * kBlock) >> l2, nj = n / JB, nz = G.g / nj, KB = n / nz;
    const int jb = G.b % nj, zr = G.b / nj;
    const int j = jb * JB + ((4 * (int)threadIdx.x) >> l2), i0 = (4 * (int)threadIdx.x) & msk;
    const int jm = (j - 1) & msk, jp = (j + 1) & msk, k0 = zr * KB;
    D4 zm = zero4, own = zero4;
    if (!cold) {
      zm = P4(nat_idx(n, i0, j, (k0 - 1) & msk));
      own = P4(nat_idx(n, i0, j, k0));
    }
    for (int kk = 0; kk < KB; kk++) {
      const int k = k0 + kk;
      D4 zp = zero4, ym = zero4, yp = zero4;
      if (!cold) {
        zp = P4(nat_idx(n, i0, j, (k + 1) & msk));
        ym = P4(nat_idx(n, i0, jm, k));
        yp = P4(nat_idx(n, i0, jp, k));
      }
      const int t = ((k << l2) + j) * n + i0;
      double xl, xr;
      xlr(t, i0, &xl, &xr);
      point4(t, i0, j, k, own, ym, yp, zm, zp, xl, xr);
      zm = own;
      own = zp;
    }
  } else {
    // four consecutive points of one row per thread
    march4(G, n, [&](int t) {
      const int i0 = t & msk, j = (t >> l2) & msk, k = t >> (2 * l2);
      if (cold) {
        point4(t, i0, j, k, zero4, zero4, zero4, zero4, zero4, 0.0, 0.0);
        return;
      }
      const int rym = nat_idx(n, 0, (j - 1) & msk, k), ryp = nat_idx(n, 0, (j + 1) & msk, k);
      const int rzm = nat_idx(n, 0, j, (k - 1) & msk), rzp = nat_idx(n, 0, j, (k + 1) & msk);
      double xl, xr;
      xlr(t, i0, &xl, &xr);
      point4(t, i0, j, k, P4(t), P4(rym + i0), P4(ryp + i0), P4(rzm + i0), P4(rzp + i0), xl, xr);
    });
  }
  double bs = block_sum(sv, sh);
  double bm = block_max(qmax, sh);
  put_partials(partial, A.nbp, G, bs, bm);
}

// One workgroup: mean of sigma_p, max|q^s|, threshold; opens the step's solve.
struct FinSigma {
  struct Args {
    int nb, n3, tol_mode;
    double tol;
    const double* partial;
    Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void FinSigma::run(const Args& A, Grid) {
  const int nb = A.nb, n3 = A.n3, tol_mode = A.tol_mode;
  const double tol = A.tol;
  const double* __restrict__ partial = A.partial;
  Ctl* ctl = A.ctl;
  __shared__ double sh[kBlock / 64];
  const double tot = reduce_partials_sum(partial, nb, sh);
  const double mx = reduce_partials_max(partial + nb, nb, sh);
  if (threadIdx.x == 0) {
    ctl->mean_sigma = tot / (double)n3;
    ctl->norm_qs = mx;
    ctl->thresh = tol_mode == 0 ? tol * mx : tol;
    ctl->done = 0;
    ctl->cycles = 0;
    ctl->status = 0;
    ctl->final_buf = 0;
    ctl->pending = 0;
  }
}

// ---------------------------------------------------------------------------
// Outer residual in FP64 (Eq. 26) for M y = sigma_p, recomputed from y
// every cycle: cycle 0 forms r = (sigma_p - mean) - M y from the predicted
// multiplier; cycle c > 0 first applies the V-cycle correction, y += e in
// FP64, and forms the same residual from the new y.  The multiplier
// ping-pongs between y0 (cycles 0, 2, ...) and y1 (cycles 1, 3, ...), since
// every point reads its neighbours' old values; the control block's
// final_buf names the buffer of the last cycle.  r goes to the next V-cycle
// in precision T, colour-split; the finalize pass records the residual, the
// running mean of y and the stop decision.
// ---------------------------------------------------------------------------
template <typename T>
struct OuterArgs {
  int n, first;
  const double* sigma;
  double *y0, *y1;
  const T *e0, *e1;
  T *r0, *r1;
  double* partial;
  Ctl* ctl;
  // first residual of a single system: sigma's partials (null: the
  // control block already holds the step's mean, FinSigma)
  const double* spart;
  int tol_mode;
  double tol;
  int nbp;   // partial stride of this launch and of sigma's (>= the grid)
};
// NT > kBlock: the shared-row column walk (n >= 256)
template <typename T, int NT = kBlock>
struct Outer {
  using Args = OuterArgs<T>;
  static constexpr int kThreads = NT;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int NT>
__device__ void Outer<T, NT>::run(const Args& A, Grid G) {
  const int n = A.n, first = A.first;
  const double* __restrict__ sigma = A.sigma;
  const T* __restrict__ e0 = A.e0;
  const T* __restrict__ e1 = A.e1;
  T* __restrict__ r0 = A.r0;
  T* __restrict__ r1 = A.r1;
  double* __restrict__ partial = A.partial;
  Ctl* ctl = A.ctl;
  __shared__ double sh[NT / 64];
  __shared__ double s_mean;
  const CsGeo g(n);
  const int n3 = n * n * n, msk = n - 1;
  double mean_sigma;
  if (first && A.spart) {
    // FinSigma's reduction in every workgroup (same split and tree, so the
    // same mean); the first workgroup opens the step's solve in the control
    // block
    const int snb = A.nbp;
    const double tot = reduce_partials_sum(A.spart, snb, sh);
    const double mx = reduce_partials_max(A.spart + snb, snb, sh);
    if (threadIdx.x == 0) {
      s_mean = tot / (double)n3;
      if (G.b == 0) {
        ctl->mean_sigma = s_mean;
        ctl->norm_qs = mx;
        ctl->thresh = A.tol_mode == 0 ? A.tol * mx : A.tol;
        ctl->done = 0;
        ctl->cycles = 0;
        ctl->status = 0;
        ctl->final_buf = 0;
      }
    }
    __syncthreads();
    mean_sigma = s_mean;
  } else {
    if (ctl->done) return;
    mean_sigma = ctl->mean_sigma;
  }
  const int c = first ? 0 : ctl->cycles + 1;
  double rmax = 0.0, ysum = 0.0;
  // Correction e at four consecutive points x = i0 .. i0+3 of row (j, k):
  // their colours alternate, so each colour array holds two of them side
  // by side (x = i0, i0+2 in the array of colour par, x = i0+1, i0+3 in the
  // other).
  auto E4 = [&](int j, int k, int i0, D4* out) {
    const int par = (i0 + j + k) & 1;
    const int idx = cs_index(g, i0, j, k);
    const T* a = par ? e1 : e0;
    const T* b = par ? e0 : e1;
    const T a0 = a[idx], a1 = a[idx + 1], b0 = b[idx], b1 = b[idx + 1];
    out->v[0] = (double)a0;
    out->v[1] = (double)b0;
    out->v[2] = (double)a1;
    out->v[3] = (double)b1;
  };
  auto E1 = [&](int x, int j, int k) -> double {
    return (double)(((x + j + k) & 1) ? e1 : e0)[cs_index(g, x, j, k)];
  };
  // y of cycle c on four consecutive points of a row: the stored y (cycle
  // 0), or the previous cycle's y plus this cycle's correction
  const double* yo = (c & 1) ? A.y0 : A.y1;   // cycle c - 1 (cycle 0: the predictor in y0)
  const double* ys = c == 0 ? A.y0 : yo;
  auto Y4 = [&](int i0, int j, int k) {
    D4 v = ld4(ys, nat_idx(n, i0, j, k));
    if (c > 0) {
      D4 e;
      E4(j, k, i0, &e);
#pragma unroll
      for (int q = 0; q < 4; q++) v.v[q] += e.v[q];
    }
    return v;
  };
  auto Y1 = [&](int x, int j, int k) {
    double v = ys[nat_idx(n, x, j, k)];
    if (c > 0) v += E1(x, j, k);
    return v;
  };
  // residual and new y of the four points at (i0.., j, k) from the y rows
  // of the point, its y and z neighbours and the x-neighbours xl, xr of its
  // first and last point; stores y (c > 0) and r
  auto point4 = [&](int t, int i0, int j, int k, const D4& own, const D4& ym, const D4& yp, const D4& zm,
                    const D4& zp, double xl, double xr) {
    double r[4], yv[4];
    const D4 sg = ld4(sigma, t);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const double xm = q == 0 ? xl : own.v[q - 1], xp = q == 3 ? xr : own.v[q + 1];
      const double nb = ((xm + xp) + (ym.v[q] + yp.v[q])) + (zm.v[q] + zp.v[q]);
      yv[q] = own.v[q];
      r[q] = (sg.v[q] - mean_sigma) - (nb - 6.0 * own.v[q]);
    }
    if (c > 0) st4((c & 1) ? A.y1 : A.y0, t, yv);
    {
      // r in precision T, colour-split, in the pattern of E4
      const int par = (i0 + j + k) & 1;
      const int idx = cs_index(g, i0, j, k);
      T* a = par ? r1 : r0;
      T* b = par ? r0 : r1;
      a[idx] = (T)r[0];
      b[idx] = (T)r[1];
      a[idx + 1] = (T)r[2];
      b[idx + 1] = (T)r[3];
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      rmax = fmax(rmax, fabs(r[q]));
      ysum += yv[q];
    }
  };
  if constexpr (NT > kBlock) {
    extern __shared__ __align__(16) double col_lds[];
    col_walk<NT>(G, n, col_lds, Y4,
                 [&](int t, int i0, int j, int k, const D4& own, const D4& ym, const D4& yp, const D4& zm,
                     const D4& zp, double xl, double xr) { point4(t, i0, j, k, own, ym, yp, zm, zp, xl, xr); });
  } else if (n >= 64) {
    // the column walk of march4, with the z-neighbour rows kept in
    // registers from plane to plane: each plane loads only its z+1 row and
    // its y-neighbour rows (shared through the XCD's L2 with the workgroups
    // of the adjacent rows)
    const int JB = (4 * kBlock) >> g.l2, nj = n / JB, nz = G.g / nj, KB = n / nz;
    const int jb = G.b % nj, zr = G.b / nj;
    const int j = jb * JB + ((4 * (int)threadIdx.x) >> g.l2), i0 = (4 * (int)threadIdx.x) & msk;
    const int jm = (j - 1) & msk, jp = (j + 1) & msk, k0 = zr * KB;
    D4 zm = Y4(i0, j, (k0 - 1) & msk), own = Y4(i0, j, k0);
    for (int kk = 0; kk < KB; kk++) {
      const int k = k0 + kk;
      const D4 zp = Y4(i0, j, (k + 1) & msk);
      const D4 ym = Y4(i0, jm, k), yp = Y4(i0, jp, k);
      point4(((k << g.l2) + j) * n + i0, i0, j, k, own, ym, yp, zm, zp, Y1((i0 - 1) & msk, j, k),
             Y1((i0 + 4) & msk, j, k));
      zm = own;
      own = zp;
    }
  } else {
    // four consecutive points of one row per thread
    march4(G, n, [&](int t) {
      const int i0 = t & msk, j = (t >> g.l2) & msk, k = t >> (2 * g.l2);
      const int jm = (j - 1) & msk, jp = (j + 1) & msk, km = (k - 1) & msk, kp = (k + 1) & msk;
      point4(t, i0, j, k, Y4(i0, j, k), Y4(i0, jm, k), Y4(i0, jp, k), Y4(i0, j, km), Y4(i0, j, kp),
             Y1((i0 - 1) & msk, j, k), Y1((i0 + 4) & msk, j, k));
    });
  }
  double bm = block_max(rmax, sh);
  double bs = block_sum(ysum, sh);
  put_partials(partial, A.nbp, G, bm, bs);
  if (threadIdx.x == 0 && G.b == 0) ctl->pending = c + 1;
}

// ---------------------------------------------------------------------------
// Fourth-order (Hermitian, Mehrstellen) discretisation, the higher-order
// option the paper mentions after Eq. 21: the constraint becomes
// A phi = -(4 pi / h) B q^s with the 19-point operator
// A = (1/6)(2 sum_faces + sum_edges - 24) and B = (1/12)(sum_faces + 6), so
// sigma_p = (h/4pi) A phi_p + B q^s and the outer residual is
// r = sigma_p - mean - A y.  The V-cycle keeps the seven-point operator:
// each cycle is a defect-correction step, which converges because A and M
// agree on the smooth modes the Gaussian-smoothed charge carries.  These
// kernels handle one point at a time with direct neighbour loads (the
// seven-point kernels are the tuned path); their grids and partials match
// Sigma / Outer, so the stop decisions are made the same way.
// ---------------------------------------------------------------------------
// v at (i, j, k) + the sums of its 6 face and 12 edge neighbours.
template <typename F>
__device__ __forceinline__ void stencil19(int n, int i, int j, int k, F v, double* c, double* faces, double* edges) {
  const int msk = n - 1;
  const int im = (i - 1) & msk, ip = (i + 1) & msk, jm = (j - 1) & msk, jp = (j + 1) & msk;
  const int km = (k - 1) & msk, kp = (k + 1) & msk;
  *c = v(i, j, k);
  *faces = ((v(im, j, k) + v(ip, j, k)) + (v(i, jm, k) + v(i, jp, k))) + (v(i, j, km) + v(i, j, kp));
  *edges = (v(im, jm, k) + v(ip, jm, k) + v(im, jp, k) + v(ip, jp, k)) +
           (v(im, j, km) + v(ip, j, km) + v(im, j, kp) + v(ip, j, kp)) +
           (v(i, jm, km) + v(i, jp, km) + v(i, jm, kp) + v(i, jp, kp));
}

template <typename TQ>
struct SigmaHO {
  using Args = SigmaArgs<TQ>;
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    const int n = A.n, msk = n - 1, l2 = __builtin_ctz(n);
    const double h = A.h;
    const Ctl* ctl = A.ctl;
    __shared__ double sh[kBlock / 64];
    const int cold = ctl->cold, m_eff = ctl->m_eff;
    const double* pk = ctl->k_idx ? A.phi1 : A.phi0;
    const double* pkm1 = ctl->k_idx ? A.phi0 : A.phi1;
    const double* const yb[3] = {A.yb0, A.yb1, A.yb2};
    const double* y0 = yb[ctl->yh0];
    const double* y1 = yb[ctl->yh1];
    const double* y2 = yb[ctl->yh2];
    double sv = 0.0, qmax = 0.0;
    auto Q = [&](int x, int y, int z) { return (double)A.qs[nat_idx(n, x, y, z)]; };
    auto P = [&](int x, int y, int z) {
      const int a = nat_idx(n, x, y, z);
      return 2.0 * pk[a] - pkm1[a];
    };
    march4(G, n, [&](int t) {
      const int i0 = t & msk, j = (t >> l2) & msk, k = t >> (2 * l2);
      double sg[4], yv[4];
      for (int q = 0; q < 4; q++) {
        const int i = i0 + q, a = t + q;
        double qc, qf, qe;
        stencil19(n, i, j, k, Q, &qc, &qf, &qe);
        const double bq = (qf + 6.0 * qc) / 12.0;
        double v = bq;
        if (!cold) {
          double pc, pf, pe;
          stencil19(n, i, j, k, P, &pc, &pf, &pe);
          v = h / (4.0 * kPi) * ((2.0 * pf + pe - 24.0 * pc) / 6.0) + bq;
        }
        sg[q] = v;
        double yy = 0.0;
        if (m_eff == 1) yy = y0[a];
        else if (m_eff == 2) yy = 2.0 * y0[a] - y1[a];
        else if (m_eff == 3) yy = 3.0 * y0[a] - 3.0 * y1[a] + y2[a];
        yv[q] = yy;
        sv += v;
        qmax = fmax(qmax, fabs(qc));
      }
      st4(A.sigma, t, sg);
      st4(A.y, t, yv);
    });
    double bs = block_sum(sv, sh);
    double bm = block_max(qmax, sh);
    put_partials(A.partial, A.nbp, G, bs, bm);
  }
};

template <typename T>
struct OuterHO {
  using Args = OuterArgs<T>;
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    const int n = A.n, first = A.first, msk = n - 1, l2 = __builtin_ctz(n);
    Ctl* ctl = A.ctl;
    __shared__ double sh[kBlock / 64];
    __shared__ double s_mean;
    const CsGeo g(n);
    const int n3 = n * n * n;
    double mean_sigma;
    if (first && A.spart) {
      const int snb = A.nbp;
      const double tot = reduce_partials_sum(A.spart, snb, sh);
      const double mx = reduce_partials_max(A.spart + snb, snb, sh);
      if (threadIdx.x == 0) {
        s_mean = tot / (double)n3;
        if (G.b == 0) {
          ctl->mean_sigma = s_mean;
          ctl->norm_qs = mx;
          ctl->thresh = A.tol_mode == 0 ? A.tol * mx : A.tol;
          ctl->done = 0;
          ctl->cycles = 0;
          ctl->status = 0;
          ctl->final_buf = 0;
        }
      }
      __syncthreads();
      mean_sigma = s_mean;
    } else {
      if (ctl->done) return;
      mean_sigma = ctl->mean_sigma;
    }
    const int c = first ? 0 : ctl->cycles + 1;
    const double* yo = (c & 1) ? A.y0 : A.y1;
    const double* ys = c == 0 ? A.y0 : yo;
    // y of cycle c: the stored y (cycle 0) or the previous y plus this cycle's correction
    auto Y = [&](int x, int y, int z) {
      double v = ys[nat_idx(n, x, y, z)];
      if (c > 0) v += (double)(((x + y + z) & 1) ? A.e1 : A.e0)[cs_index(g, x, y, z)];
      return v;
    };
    double rmax = 0.0, ysum = 0.0;
    march4(G, n, [&](int t) {
      const int i0 = t & msk, j = (t >> l2) & msk, k = t >> (2 * l2);
      double yv[4];
      for (int q = 0; q < 4; q++) {
        const int i = i0 + q;
        double yc, yf, ye;
        stencil19(n, i, j, k, Y, &yc, &yf, &ye);
        const double r = (A.sigma[t + q] - mean_sigma) - (2.0 * yf + ye - 24.0 * yc) / 6.0;
        yv[q] = yc;
        (((i + j + k) & 1) ? A.r1 : A.r0)[cs_index(g, i, j, k)] = (T)r;
        rmax = fmax(rmax, fabs(r));
        ysum += yc;
      }
      if (c > 0) st4((c & 1) ? A.y1 : A.y0, t, yv);
    });
    double bm = block_max(rmax, sh);
    double bs = block_sum(ysum, sh);
    put_partials(A.partial, A.nbp, G, bm, bs);
    if (threadIdx.x == 0 && G.b == 0) ctl->pending = c + 1;
  }
};

// The stop decision's two reductions over the outer residual's partials
// (max of the first nb, sum of the next nb) with the split and tree of a
// 1024-thread workgroup: virtual thread v folds partials v, v + 1024, ...,
// each 64-lane group reduces by butterfly, and the 16 group results are
// combined in order.  Any workgroup of a power-of-two multiple of 64 threads
// computes it, so every place the decision is made gives the same bits.
// sh: 32 doubles.  Results valid in thread 0.
__device__ __forceinline__ void decide_reduce(const double* __restrict__ partial, int nb, double* sh, double* res,
                                              double* ys) {
  constexpr int kV = 1024;
  const int nt = blockDim.x, lane = threadIdx.x & 63;
  for (int v0 = 0; v0 < kV; v0 += nt) {
    const int v = v0 + threadIdx.x;
    double m = 0.0, s = 0.0;
    for (int i = v; i < nb; i += kV) {
      m = fmax(m, partial[i]);
      s += partial[nb + i];
    }
    m = wave_max(m);
    s = wave_sum(s);
    if (lane == 0) {
      sh[v >> 6] = m;
      sh[16 + (v >> 6)] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < 16; i++) {
      a = fmax(a, sh[i]);
      b += sh[16 + i];
    }
    *res = a;
    *ys = b;
  }
}

// The state the field update needs from the stop decision.
struct DecideOut {
  int done, final_buf;
  double mean_y;
};

// The stop decision of the pending outer residual: residual of cycle c (max
// norm), running mean of y, cycle count, which buffer holds y, done/status.
// The partials are read while the pending mark is still in flight.  Every
// thread of the workgroup gets the outcome in *out (shared); only a writer
// workgroup records it in the control block, and clears the pending mark if
// `clear`.  A launch whose workgroups all decide (the field update) must not
// clear it: a workgroup that started later would see no decision pending and
// take fields the writer may not have stored yet; the decision is idempotent,
// so a later decision point may repeat it.  With nothing pending the outcome
// is the control block's current state.
__device__ __forceinline__ void outer_decide(Ctl* ctl, const double* __restrict__ partial, int nb, int n3,
                                             int max_cycles, bool writer, bool clear, double* sh, DecideOut* out) {
  const int pend = ctl->pending;
  double res = 0.0, ys = 0.0;
  decide_reduce(partial, nb, sh, &res, &ys);
  if (threadIdx.x == 0) {
    if (pend) {
      const int c = pend - 1;
      int done = ctl->done;
      const double mean_y = ys / (double)n3;
      int status = 0;
      if (res <= ctl->thresh) {
        done = 1;
      } else if (c >= max_cycles) {
        done = 1;
        status = 1;
      }
      if (writer) {
        ctl->res_hist[c] = res;
        ctl->mean_y = mean_y;
        ctl->cycles = c;
        ctl->final_buf = c & 1;
        if (status) ctl->status = 1;
        ctl->done = done;
        if (clear) ctl->pending = 0;
      }
      *out = DecideOut{done, c & 1, mean_y};
    } else {
      *out = DecideOut{ctl->done, ctl->final_buf, ctl->mean_y};
    }
  }
  __syncthreads();
}

// The stop decision as a launch of its own (batched systems decide right
// after every residual).
struct FinOuter {
  struct Args {
    int max_cycles, nb, n3;
    const double* partial;
    Ctl* ctl;
  };
  static constexpr int kThreads = 1024;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void FinOuter::run(const Args& A, Grid) {
  __shared__ double sh[32];
  __shared__ DecideOut out;
  outer_decide(A.ctl, A.partial, A.nb, A.n3, A.max_cycles, true, true, sh, &out);
}

// ---------------------------------------------------------------------------
// V-cycle kernels on colour-split storage.  A thread owns index t of a
// colour array: m = t % (n/2), row (j,k) = t / (n/2), and the point of
// colour c is i = 2m + ((c+j+k)&1).  All neighbours of a point have the
// other colour: x-neighbours at (i+-1)/2 of the same row, y/z neighbours at
// the same m of the adjacent rows, i.e. at t +- n/2 and t +- n^2/2.  Every
// level has a power-of-two edge, so indices are shifts and masks.
// ---------------------------------------------------------------------------
// Sum of the six neighbours (other colour array o) of the point at
// colour-split index t with x = 2m + s in row (j,k), in the fixed order
// ((x- + x+) + (y- + y+)) + (z- + z+).
template <typename T>
__device__ __forceinline__ T cs_nbr6(const T* __restrict__ o, const CsGeo& g, int t, int m, int j, int k, int s) {
  const int row = t - m;
  const int xm = s ? m : (m == 0 ? g.hn - 1 : m - 1);
  const int xp = s ? (m + 1 == g.hn ? 0 : m + 1) : m;
  const int ym = j == 0 ? t + (g.n - 1) * g.hn : t - g.hn;
  const int yp = j == g.n - 1 ? t - (g.n - 1) * g.hn : t + g.hn;
  const int zm = k == 0 ? t + (g.n - 1) * g.plane : t - g.plane;
  const int zp = k == g.n - 1 ? t - (g.n - 1) * g.plane : t + g.plane;
  return ((o[row + xm] + o[row + xp]) + (o[ym] + o[yp])) + (o[zm] + o[zp]);
}

// Vector width of the half-sweeps: 16-byte accesses (4 floats, 2 doubles).
// Every level a half-sweep runs on has n/2 divisible by 4, so a vector never
// crosses a row.
template <typename T> struct Vec;
template <> struct Vec<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int W = 2; };
template <typename T> __device__ __forceinline__ T vget(const typename Vec<T>::type& v, int q);
template <> __device__ __forceinline__ float vget<float>(const float4& v, int q) {
  return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
}
template <> __device__ __forceinline__ double vget<double>(const double2& v, int q) { return q == 0 ? v.x : v.y; }
template <typename T> __device__ __forceinline__ void vset(typename Vec<T>::type& v, int q, T x);
template <> __device__ __forceinline__ void vset<float>(float4& v, int q, float x) {
  if (q == 0) v.x = x; else if (q == 1) v.y = x; else if (q == 2) v.z = x; else v.w = x;
}
template <> __device__ __forceinline__ void vset<double>(double2& v, int q, double x) {
  if (q == 0) v.x = x; else v.y = x;
}

// -x/6 rounded on its own.  The first sweep from e = 0 sums red values -r/6
// that it computes on the fly; without contraction they are exactly the
// values a stored red array would hold, so the sweep's black result does not
// depend on whether the reds come from memory or are recomputed.
template <typename T>
__device__ __forceinline__ T neg_sixth(T x) {
#pragma clang fp contract(off)
  return -x * T(1.0 / 6.0);
}

// Speculative start of the small V-cycle launches: the control block's stop
// flag and the operands are loaded together and the flag is tested just
// before the first store, so the two memory round trips of a launch that
// moves little data overlap.  keep_issued() makes the computed value live
// before that test (the compiler may not defer the loads past it).  Large
// levels and batched launches test the flag first instead, so converged
// systems read nothing.
__device__ __forceinline__ void keep_issued(float v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep_issued(double v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep_issued(const float4& v) {
  asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}
__device__ __forceinline__ void keep_issued(const double2& v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }

// cs_nbr6 for the W points t..t+W-1 of one row (same colour, same x-parity
// s), each neighbour value passed through f first.  x-neighbours come from
// the row's own vector plus one edge element, y/z neighbours from the vectors
// at t +- n/2 and t +- n^2/2; per point the sum order is that of cs_nbr6.
template <typename T, typename F>
__device__ __forceinline__ void cs_nbr6_vec(const T* __restrict__ o, const CsGeo& g, int t, int m, int j, int k,
                                            int s, F f, T* out) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const int row = t - m;
  const V own = *reinterpret_cast<const V*>(o + t);
  const T edge = f(s ? o[row + (m + W == g.hn ? 0 : m + W)] : o[row + (m == 0 ? g.hn - 1 : m - 1)]);
  const int ym = j == 0 ? t + (g.n - 1) * g.hn : t - g.hn;
  const int yp = j == g.n - 1 ? t - (g.n - 1) * g.hn : t + g.hn;
  const int zm = k == 0 ? t + (g.n - 1) * g.plane : t - g.plane;
  const int zp = k == g.n - 1 ? t - (g.n - 1) * g.plane : t + g.plane;
  const V vym = *reinterpret_cast<const V*>(o + ym), vyp = *reinterpret_cast<const V*>(o + yp);
  const V vzm = *reinterpret_cast<const V*>(o + zm), vzp = *reinterpret_cast<const V*>(o + zp);
#pragma unroll
  for (int q = 0; q < W; q++) {
    const T xm = s ? f(vget<T>(own, q)) : (q == 0 ? edge : f(vget<T>(own, q - 1)));
    const T xp = s ? (q == W - 1 ? edge : f(vget<T>(own, q + 1))) : f(vget<T>(own, q));
    out[q] = ((xm + xp) + (f(vget<T>(vym, q)) + f(vget<T>(vyp, q)))) + (f(vget<T>(vzm, q)) + f(vget<T>(vzp, q)));
  }
}

// Kernels below carry a FIN template flag that is 1 only on the finest level,
// so profiles report the finest-level instances under their own names.

// First pre-smoothing sweep from e = 0: red = -r/6, then black from those reds
// (one thread per W consecutive points of a row).
template <typename T, int FIN, int SPEC>
struct SweepZero {
  struct Args {
    int n;
    const T *r0, *r1;
    T *e0, *e1;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN, int SPEC>
__device__ void SweepZero<T, FIN, SPEC>::run(const Args& A, Grid G) {
  const int n = A.n;
  const T* __restrict__ r0 = A.r0;
  const T* __restrict__ r1 = A.r1;
  T* __restrict__ e0 = A.e0;
  T* __restrict__ e1 = A.e1;
  const int done = A.ctl->done;
  if (!SPEC && done) return;
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const CsGeo g(n);
  const int half = n * g.hn * n;
  const int t = (G.b * kBlock + threadIdx.x) * W;
  if (t >= half) return;
  int m, j, k;
  cs_decode(g, t, &m, &j, &k);
  const T sixth = T(1.0 / 6.0);
  const V rr = *reinterpret_cast<const V*>(r0 + t);
  V er;
#pragma unroll
  for (int q = 0; q < W; q++) vset<T>(er, q, neg_sixth(vget<T>(rr, q)));
  // black points of the same row: their neighbours are the red values -r0/6
  T nb[W];
  cs_nbr6_vec(r0, g, t, m, j, k, (1 + j + k) & 1, [](T x) { return neg_sixth(x); }, nb);
  const V rb = *reinterpret_cast<const V*>(r1 + t);
  V eb;
#pragma unroll
  for (int q = 0; q < W; q++) vset<T>(eb, q, (nb[q] - vget<T>(rb, q)) * sixth);
  if (SPEC) {
    keep_issued(eb);
    if (done) return;
  }
  *reinterpret_cast<V*>(e0 + t) = er;
  *reinterpret_cast<V*>(e1 + t) = eb;
}

template <typename T, int FIN, int SPEC>
struct Halfsweep {
  struct Args {
    int n, colour;
    T* ec;
    const T *eo, *rc;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN, int SPEC>
__device__ void Halfsweep<T, FIN, SPEC>::run(const Args& A, Grid G) {
  const int n = A.n, colour = A.colour;
  T* __restrict__ ec = A.ec;
  const T* __restrict__ eo = A.eo;
  const T* __restrict__ rc = A.rc;
  const int done = A.ctl->done;
  if (!SPEC && done) return;
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const CsGeo g(n);
  const int half = n * g.hn * n;
  const int t = (G.b * kBlock + threadIdx.x) * W;
  if (t >= half) return;
  int m, j, k;
  cs_decode(g, t, &m, &j, &k);
  T nb[W];
  cs_nbr6_vec(eo, g, t, m, j, k, (colour + j + k) & 1, [](T x) { return x; }, nb);
  const V r = *reinterpret_cast<const V*>(rc + t);
  V out;
#pragma unroll
  for (int q = 0; q < W; q++) vset<T>(out, q, (nb[q] - vget<T>(r, q)) * T(1.0 / 6.0));
  if (SPEC) {
    keep_issued(out);
    if (done) return;
  }
  *reinterpret_cast<V*>(ec + t) = out;
}

// Residual rho = r - M e at the 27 fine points around 2I, full weighting,
// times 4 (coarse operator rediscretised on 2h).  One thread per coarse point.
// When the last pre-smoothing operation was a black half-sweep, the black
// residuals are zero up to rounding (Gauss-Seidel just solved those rows), so
// only the 13 red points of the 27-point stencil are evaluated (red_only).
template <typename T, int FIN, int SPEC>
struct ResidRestrict {
  struct Args {
    int n, red_only;
    const T *e0, *e1, *r0, *r1;
    T *rc0, *rc1;
    const Ctl* ctl;
  };
  // one thread per coarse point: small workgroups spread the few coarse
  // points of the upper-middle levels over every compute unit
  static constexpr int kThreads = 64;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN, int SPEC>
__device__ void ResidRestrict<T, FIN, SPEC>::run(const Args& A, Grid G) {
  const int n = A.n, red_only = A.red_only;
  const T* __restrict__ e0 = A.e0;
  const T* __restrict__ e1 = A.e1;
  const T* __restrict__ r0 = A.r0;
  const T* __restrict__ r1 = A.r1;
  T* __restrict__ rc0 = A.rc0;
  T* __restrict__ rc1 = A.rc1;
  const int done = A.ctl->done;
  if (!SPEC && done) return;
  const CsGeo g(n), gc(n >> 1);
  const int nc = gc.n;
  const int t = G.b * kThreads + threadIdx.x;
  if (t >= nc * nc * nc) return;
  const int I = t & (nc - 1), J = (t >> gc.l2) & (nc - 1), K = t >> (2 * gc.l2);
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  const int msk = n - 1;
  T s = T(0);
  for (int c = -1; c <= 1; c++) {
    const int z = (2 * K + c) & msk;
    for (int b = -1; b <= 1; b++) {
      const int y = (2 * J + b) & msk;
      T row = T(0);
      for (int a = -1; a <= 1; a++) {
        const int x = (2 * I + a) & msk;
        const int odd = (x + y + z) & 1;
        if (red_only && odd) continue;
        const int ti = cs_index(g, x, y, z);
        const T ev = odd ? e1[ti] : e0[ti];
        const T rv = odd ? r1[ti] : r0[ti];
        const T rho = rv - (cs_nbr6(odd ? e0 : e1, g, ti, x >> 1, y, z, x & 1) - T(6) * ev);
        row += wt[a + 1] * rho;
      }
      s += wt[b + 1] * wt[c + 1] * row;
    }
  }
  const T v = T(4) * s;
  if (SPEC) {
    keep_issued(v);
    if (done) return;
  }
  T* out = ((I + J + K) & 1) ? rc1 : rc0;
  out[cs_index(gc, I, J, K)] = v;
}

// Full weighting x 4 at the coarse points I0 .. I0+W-1 of coarse row (J,K),
// the red residuals r - M e of the 9 fine rows formed on the fly (the black
// ones vanish after a black half-sweep), in the order of ResidRestrict.
// ROWS_UNROLL: how far the 3 x 3 row loop is unrolled (3 for the separate
// launch; 1 inside the tail, whose 1024-thread workgroup has fewer registers).
template <typename T, int ROWS_UNROLL>
__device__ __forceinline__ void restrict_red_recompute(const T* e0, const T* e1, const T* r0, const CsGeo& g, int I0,
                                                       int J, int K, T* v) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  const int msk = g.n - 1, nc = g.hn;
  T s[W];
#pragma unroll
  for (int q = 0; q < W; q++) s[q] = T(0);
#pragma unroll ROWS_UNROLL
  for (int c = -1; c <= 1; c++) {
    const int z = (2 * K + c) & msk;
#pragma unroll ROWS_UNROLL
    for (int b = -1; b <= 1; b++) {
      const int y = (2 * J + b) & msk;
      const int par = (y + z) & 1;   // red points of this row sit at x = 2m + par
      const int row0 = ((z << g.l2) + y) << (g.l2 - 1);
      const int tv = row0 + I0;
      T nb[W];
      cs_nbr6_vec(e1, g, tv, I0, y, z, par, [](T x) { return x; }, nb);
      const V ev = *reinterpret_cast<const V*>(e0 + tv);
      const V rv = *reinterpret_cast<const V*>(r0 + tv);
      T rho[W];
#pragma unroll
      for (int q = 0; q < W; q++) rho[q] = vget<T>(rv, q) - (nb[q] - T(6) * vget<T>(ev, q));
      const T wbc = wt[b + 1] * wt[c + 1];
      if (par == 0) {
        // only x = 2I is red: m = I
#pragma unroll
        for (int q = 0; q < W; q++) {
          T row = T(0);
          row += wt[1] * rho[q];
          s[q] += wbc * row;
        }
      } else {
        // x = 2I - 1 (m = I - 1) and x = 2I + 1 (m = I)
        const int me = (I0 - 1) & (nc - 1);
        const int te = row0 + me;
        const T rho_e = r0[te] - (cs_nbr6(e1, g, te, me, y, z, 1) - T(6) * e0[te]);
#pragma unroll
        for (int q = 0; q < W; q++) {
          T row = T(0);
          row += wt[0] * (q == 0 ? rho_e : rho[q - 1]);
          row += wt[2] * rho[q];
          s[q] += wbc * row;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < W; q++) v[q] = T(4) * s[q];
}

// ResidRestrict for red_only, W = Vec<T>::W consecutive coarse points of a
// coarse row per thread: the red residuals of each of the 9 fine rows are
// formed as one row vector (the neighbour sums of a half-sweep) plus, in rows
// whose red points sit at odd x, the one residual left of the vector; every
// coarse point then sums its 13 red terms in the order of ResidRestrict, so
// the results are those of the one-point-per-thread kernel.
template <typename T, int FIN, int SPEC>
struct RestrictRed {
  using Args = typename ResidRestrict<T, FIN, SPEC>::Args;
  static constexpr int kThreads = 64;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN, int SPEC>
__device__ void RestrictRed<T, FIN, SPEC>::run(const Args& A, Grid G) {
  constexpr int W = Vec<T>::W;
  const int n = A.n;
  const T* __restrict__ e0 = A.e0;
  const T* __restrict__ e1 = A.e1;
  const T* __restrict__ r0 = A.r0;
  const int done = A.ctl->done;
  if (!SPEC && done) return;
  const CsGeo g(n), gc(n >> 1);
  const int nc = gc.n;
  const int t = (G.b * kThreads + threadIdx.x) * W;
  if (t >= nc * nc * nc) return;
  const int I0 = t & (nc - 1), J = (t >> gc.l2) & (nc - 1), K = t >> (2 * gc.l2);
  T v[W];
  restrict_red_recompute<T, 3>(e0, e1, r0, g, I0, J, K, v);
  if (SPEC) {
    keep_issued(v[W - 1]);
    if (done) return;
  }
#pragma unroll
  for (int q = 0; q < W; q++) {
    const int I = I0 + q;
    T* out = ((I + J + K) & 1) ? A.rc1 : A.rc0;
    out[cs_index(gc, I, J, K)] = v[q];
  }
}

// The red-only restriction as a column walk over fine z-planes (fine levels
// from 256^3 up, single systems).  RestrictRed recomputes every fine red
// residual for each coarse point whose 27-point stencil covers it, 3.4
// times on average, each with its own neighbour loads; here a workgroup owns
// JB coarse rows of a band of KB coarse planes and walks the fine planes
// 2 K0 - 1 .. 2 (K0 + KB) - 1 once:
//  * each thread owns W red points of one fine row (the workgroup's 2 JB
//    fine rows 2 J0 .. 2 J0 + 2 JB - 1, plus the halo row 2 J0 - 1 taken by the
//    first G_x = n / (2 W) threads) and keeps that row's black values of
//    planes z-1, z, z+1 in registers;
//  * plane z's black rows 2 J0 - 2 .. 2 J0 + 2 JB sit in LDS for the x- and
//    y-neighbours, so each fine value is loaded once per workgroup;
//  * the red residuals of plane z go to LDS, and the threads of the even
//    fine rows (one per W coarse points of coarse row J) add the plane's three
//    weighted rows to the running sums of coarse planes K (z = 2K - 1, 2K,
//    2K + 1); a coarse plane is written when its last fine plane is done.
// Per coarse point the terms are added in RestrictRed's order (planes, then
// rows, ascending), each formed with its arithmetic, so the results agree
// with it to the rounding of the contracted products.  One workgroup
// barrier per fine plane; LDS holds two buffers of each kind.
template <typename T>
struct RestrictColGeo {
  int nc, W, gx, JB, erows, rrows;
  __host__ __device__ RestrictColGeo(int n, int nt) {
    W = 16 / (int)sizeof(T);
    nc = n / 2;
    gx = nc / W;                // threads per fine row
    JB = nt / (2 * gx);         // coarse rows per workgroup
    erows = 2 * JB + 3;         // black rows 2 J0 - 2 .. 2 J0 + 2 JB
    rrows = 2 * JB + 1;         // residual rows 2 J0 - 1 .. 2 J0 + 2 JB - 1
  }
  __host__ __device__ int lds_elems() const { return 2 * (erows + rrows) * nc; }
};
constexpr int kRestrictColThreads = 512;
// Single systems (not recorded into a batch), fine levels 256^3 and 512^3.
inline bool restrict_col_on(int n) { return n >= 256 && n <= 512 && !g_recorder; }

template <typename T, int FIN>
struct RestrictCol {
  using Args = typename ResidRestrict<T, FIN, 0>::Args;
  static constexpr int kThreads = kRestrictColThreads;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN>
__device__ void RestrictCol<T, FIN>::run(const Args& A, Grid G) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  if (A.ctl->done) return;
  const int n = A.n, msk = n - 1;
  const CsGeo g(n), gc(n >> 1);
  const RestrictColGeo<T> cg(n, kThreads);
  const int nc = cg.nc, gx = cg.gx, JB = cg.JB, cmsk = nc - 1;
  const int nj = nc / JB, nz = G.g / nj, KB = nc / nz;
  const int jb = G.b % nj, zr = G.b / nj;
  const int J0 = jb * JB, K0 = zr * KB;
  const int tid = threadIdx.x;
  const int f = tid / gx, m0 = (tid % gx) * W;   // own fine row 2 J0 + f, red entries m0 .. m0 + W - 1
  const bool halo = tid < gx;                     // also the residual row 2 J0 - 1
  const bool top = tid >= gx && tid < 2 * gx;     // loads black row 2 J0 + 2 JB
  extern __shared__ __align__(16) unsigned char rcol_lds[];
  T* const ebuf = reinterpret_cast<T*>(rcol_lds);          // [2][erows][nc]
  T* const rbuf = ebuf + 2 * cg.erows * nc;                 // [2][rrows][nc]
  const T* __restrict__ e0 = A.e0;
  const T* __restrict__ e1 = A.e1;
  const T* __restrict__ r0 = A.r0;
  const int yo = (2 * J0 + f) & msk, yh = (2 * J0 - 1) & msk;
  const int yb = (2 * J0 - 2) & msk, yt = (2 * J0 + 2 * JB) & msk;
  auto at = [&](const T* a, int y, int z) {
    return *reinterpret_cast<const V*>(a + ((((z & msk) << g.l2) + y) << (g.l2 - 1)) + m0);
  };
  auto eput = [&](int buf, int ly, const V& v) {
    *reinterpret_cast<V*>(ebuf + (buf * cg.erows + ly) * nc + m0) = v;
  };
  // red residuals of W points of fine row y (LDS black row ly) at plane z
  auto rho_row = [&](int buf, int ly, int y, int z, const V& bzm, const V& bzp, T* rho) {
    const T* row = ebuf + (buf * cg.erows + ly) * nc;
    const int par = (y + z) & 1;
    const V own = *reinterpret_cast<const V*>(row + m0);
    const T edge = par ? row[(m0 + W) & cmsk] : row[(m0 - 1) & cmsk];
    const V vym = *reinterpret_cast<const V*>(row - nc + m0), vyp = *reinterpret_cast<const V*>(row + nc + m0);
    const V ev = at(e0, y, z), rv = at(r0, y, z);
#pragma unroll
    for (int q = 0; q < W; q++) {
      const T xm = par ? vget<T>(own, q) : (q == 0 ? edge : vget<T>(own, q - 1));
      const T xp = par ? (q == W - 1 ? edge : vget<T>(own, q + 1)) : vget<T>(own, q);
      const T nb = ((xm + xp) + (vget<T>(vym, q) + vget<T>(vyp, q))) + (vget<T>(bzm, q) + vget<T>(bzp, q));
      rho[q] = vget<T>(rv, q) - (nb - T(6) * vget<T>(ev, q));
    }
  };
  const int zs = 2 * K0 - 1, ze = 2 * (K0 + KB) - 1;
  // black values of the own (and halo) row at planes z - 1, z, z + 1
  V om = at(e1, yo, zs - 1), oc = at(e1, yo, zs), hm{}, hc{};
  eput(0, f + 2, oc);
  if (halo) {
    hm = at(e1, yh, zs - 1);
    hc = at(e1, yh, zs);
    eput(0, 1, hc);
    eput(0, 0, at(e1, yb, zs));
  }
  if (top) eput(0, 2 * JB + 2, at(e1, yt, zs));
  __syncthreads();
  const bool coarse = (f & 1) == 0;   // threads of even fine rows: coarse row J0 + f / 2
  const int Jl = f >> 1;
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  T sk[W], sn[W];   // running sums of coarse planes K and K + 1
#pragma unroll
  for (int q = 0; q < W; q++) sk[q] = sn[q] = T(0);
  int cur = 0;
  for (int z = zs; z <= ze; z++) {
    const int nxt = cur ^ 1;
    const V op = at(e1, yo, z + 1);
    V hp{};
    if (halo) hp = at(e1, yh, z + 1);
    T rho[W];
    rho_row(cur, f + 2, yo, z, om, op, rho);
    {
      V rv;
#pragma unroll
      for (int q = 0; q < W; q++) vset<T>(rv, q, rho[q]);
      *reinterpret_cast<V*>(rbuf + (cur * cg.rrows + f + 1) * nc + m0) = rv;
    }
    if (halo) {
      T rh[W];
      rho_row(cur, 1, yh, z, hm, hp, rh);
      V rv;
#pragma unroll
      for (int q = 0; q < W; q++) vset<T>(rv, q, rh[q]);
      *reinterpret_cast<V*>(rbuf + (cur * cg.rrows) * nc + m0) = rv;
    }
    // plane z + 1's black rows for the next step
    eput(nxt, f + 2, op);
    if (halo) {
      eput(nxt, 1, hp);
      eput(nxt, 0, at(e1, yb, z + 1));
    }
    if (top) eput(nxt, 2 * JB + 2, at(e1, yt, z + 1));
    __syncthreads();
    if (coarse) {
      // fine rows 2J - 1, 2J, 2J + 1 of plane z: residual rows 2 Jl .. 2 Jl + 2
      const int cz = z & 1 ? 1 : 0;   // odd z = 2K + 1: last plane of K, first of K + 1
#pragma unroll
      for (int b = -1; b <= 1; b++) {
        const int y = (2 * (J0 + Jl) + b) & msk;
        const int par = (y + z) & 1;
        const T* rr = rbuf + (cur * cg.rrows + 2 * Jl + b + 1) * nc;
        const V rv = *reinterpret_cast<const V*>(rr + m0);
        T row[W];
        if (par == 0) {
#pragma unroll
          for (int q = 0; q < W; q++) {
            T r = T(0);
            r += wt[1] * vget<T>(rv, q);
            row[q] = r;
          }
        } else {
          const T re = rr[(m0 - 1) & cmsk];
#pragma unroll
          for (int q = 0; q < W; q++) {
            T r = T(0);
            r += wt[0] * (q == 0 ? re : vget<T>(rv, q - 1));
            r += wt[2] * vget<T>(rv, q);
            row[q] = r;
          }
        }
        if (cz) {
          if (z > zs) {
            const T w = wt[b + 1] * wt[2];
#pragma unroll
            for (int q = 0; q < W; q++) sk[q] += w * row[q];
          }
          if (z < ze) {
            const T w = wt[b + 1] * wt[0];
#pragma unroll
            for (int q = 0; q < W; q++) sn[q] += w * row[q];
          }
        } else {
          const T w = wt[b + 1] * wt[1];
#pragma unroll
          for (int q = 0; q < W; q++) sk[q] += w * row[q];
        }
      }
      if (cz) {
        if (z > zs) {
          const int K = (z - 1) >> 1, J = J0 + Jl;
#pragma unroll
          for (int q = 0; q < W; q++) {
            const int I = m0 + q;
            T* out = ((I + J + K) & 1) ? A.rc1 : A.rc0;
            out[cs_index(gc, I, J, K)] = T(4) * sk[q];
          }
        }
#pragma unroll
        for (int q = 0; q < W; q++) {
          sk[q] = sn[q];
          sn[q] = T(0);
        }
      }
    }
    om = oc;
    oc = op;
    hm = hc;
    hc = hp;
    cur = nxt;
  }
}

// The down leg of a fine level with a single pre-smoothing sweep (nu1 = 1)
// followed by black-only prolongation (nu2 >= 1), as one column walk (FP32,
// fine levels 256^3 and 512^3, single systems): the first sweep from e = 0
// (red e = -r/6, black e = (sum of its red neighbours' -r/6 - r) / 6, as
// SweepZero) and the red-only restriction of the residual it leaves (as
// RestrictCol).  Each workgroup owns JB coarse rows of a band of KB coarse
// planes and walks the fine planes; per plane z it forms the black values of
// plane z + 1 from the red residuals of planes z .. z + 2, then the red
// residuals of plane z from those black values, and adds them to the coarse
// sums.  Nothing of the red values is stored: after this restriction the
// black-only prolongation and the red half-sweep that follows overwrite
// every red value without reading it, so the red values of this sweep are
// used only here and formed on the fly.  The black values of the
// workgroup's own fine rows are written (the up leg corrects them).
// Thread rows: r0 rows 2 J0 - 3 .. 2 J0 + 2 JB + 1 (the middle plane's in
// LDS for x- and y-neighbours), of which the black rows 2 J0 - 2 .. 2 J0 +
// 2 JB are computed (in LDS for the residual's neighbours) and the
// residual rows 2 J0 - 1 .. 2 J0 + 2 JB - 1 evaluated; every value is
// computed with the arithmetic and in the order of SweepZero and
// RestrictCol, so the coarse right-hand side and the black values are
// bitwise theirs.  Two workgroup barriers per fine plane.
struct SweepRestrictGeo {
  int nc, W, gx, rows, JB;
  __host__ __device__ SweepRestrictGeo(int n, int nt) {
    W = 4;
    nc = n / 2;
    gx = nc / W;   // threads per row
    rows = nt / gx;
    JB = 1;
    while (2 * (2 * JB) + 5 <= rows && nc % (2 * JB) == 0) JB *= 2;
  }
  __host__ __device__ int r0_rows() const { return 2 * JB + 5; }
  __host__ __device__ int e1_rows() const { return 2 * JB + 3; }
  __host__ __device__ int rho_rows() const { return 2 * JB + 1; }
  __host__ __device__ int lds_floats() const { return (r0_rows() + 2 * e1_rows() + rho_rows()) * nc; }
};
constexpr int kSweepRestrictThreads = 1024;

struct SweepRestrict {
  struct Args {
    int n;
    const float *r0, *r1;
    float *e1, *rc0, *rc1;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kSweepRestrictThreads;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void SweepRestrict::run(const Args& A, Grid G) {
  using T = float;
  using V = float4;
  constexpr int W = 4;
  if (A.ctl->done) return;
  const int n = A.n, msk = n - 1;
  const CsGeo g(n), gc(n >> 1);
  const SweepRestrictGeo sg(n, kThreads);
  const int nc = sg.nc, gx = sg.gx, JB = sg.JB, cmsk = nc - 1;
  const int nj = nc / JB, nz = G.g / nj, KB = nc / nz;
  const int jb = G.b % nj, zr = G.b / nj;
  const int J0 = jb * JB, K0 = zr * KB;
  const int tid = threadIdx.x;
  const int lr0 = tid / gx, m0 = (tid % gx) * W;   // thread row: r0 row 2 J0 - 3 + lr0
  const bool r_on = lr0 < sg.r0_rows();
  const bool e_on = lr0 >= 1 && lr0 < 1 + sg.e1_rows();      // black row (LDS row lr0 - 1)
  const bool rho_on = lr0 >= 2 && lr0 < 2 + sg.rho_rows();   // residual row (LDS row lr0 - 2)
  const bool own = lr0 >= 3 && lr0 < 3 + 2 * JB;               // the workgroup's own fine row
  const int y = (2 * J0 - 3 + lr0) & msk;
  extern __shared__ __align__(16) unsigned char sr_lds[];
  T* const rbuf0 = reinterpret_cast<T*>(sr_lds);           // [r0_rows][nc]  r0 of the middle plane
  T* const ebuf = rbuf0 + sg.r0_rows() * nc;                // [2][e1_rows][nc]
  T* const hbuf = ebuf + 2 * sg.e1_rows() * nc;             // [rho_rows][nc]
  const T* __restrict__ r0 = A.r0;
  const T* __restrict__ r1 = A.r1;
  T* __restrict__ e1g = A.e1;
  auto at = [&](const T* a, int yy, int z) {
    return *reinterpret_cast<const V*>(a + ((((z & msk) << g.l2) + yy) << (g.l2 - 1)) + m0);
  };
  auto vput = [&](T* b, const V& v) { *reinterpret_cast<V*>(b + m0) = v; };
  auto neg6 = [](const V& v) { return make_float4(neg_sixth(v.x), neg_sixth(v.y), neg_sixth(v.z), neg_sixth(v.w)); };
  const int zs = 2 * K0 - 1, ze = 2 * (K0 + KB) - 1;
  const T sixth = T(1.0 / 6.0);
  // registers: r0 of planes z, z + 1 (+ z + 2 loaded each step); black of planes z - 1, z, z + 1
  // (loads run one plane ahead: r0 of plane z + 3 and r1 of plane z + 2 are
  // issued while plane z is processed)
  V rz = r_on ? at(r0, y, zs - 2) : V{}, rz1 = r_on ? at(r0, y, zs - 1) : V{};
  V rz2n = r_on ? at(r0, y, zs) : V{}, rb1n = e_on ? at(r1, y, zs - 1) : V{};
  V bm{}, bc{};
  const int cur0 = 0;
  int cur = cur0;
  const bool coarse = own && ((lr0 - 3) & 1) == 0;
  const int Jl = (lr0 - 3) >> 1;
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  T sk[W], sn[W];
#pragma unroll
  for (int q = 0; q < W; q++) sk[q] = sn[q] = T(0);
  for (int z = zs - 2; z <= ze; z++) {
    const int nxt = cur ^ 1;
    const V rz2 = rz2n, rb1 = rb1n;
    if (z < ze) {
      if (r_on) rz2n = at(r0, y, z + 3);
      if (e_on) rb1n = at(r1, y, z + 2);
    }
    if (r_on) vput(rbuf0 + lr0 * nc, rz1);   // r0 of plane z + 1
    __syncthreads();
    // black values of plane z + 1 (SweepZero's arithmetic: neighbours -r0/6)
    V bp{};
    if (e_on) {
      const T* row = rbuf0 + lr0 * nc;
      const int par = (1 + y + z + 1) & 1;   // x-parity of the black points' red neighbours
      const V o = neg6(*reinterpret_cast<const V*>(row + m0));
      const T edge = neg_sixth(par ? row[(m0 + W) & cmsk] : row[(m0 - 1) & cmsk]);
      const V vym = neg6(*reinterpret_cast<const V*>(row - nc + m0));
      const V vyp = neg6(*reinterpret_cast<const V*>(row + nc + m0));
      const V vzm = neg6(rz), vzp = neg6(rz2);
      T out[W];
#pragma unroll
      for (int q = 0; q < W; q++) {
        const T xm = par ? vget<T>(o, q) : (q == 0 ? edge : vget<T>(o, q - 1));
        const T xp = par ? (q == W - 1 ? edge : vget<T>(o, q + 1)) : vget<T>(o, q);
        const T nb = ((xm + xp) + (vget<T>(vym, q) + vget<T>(vyp, q))) + (vget<T>(vzm, q) + vget<T>(vzp, q));
        out[q] = (nb - vget<T>(rb1, q)) * sixth;
      }
      bp = make_float4(out[0], out[1], out[2], out[3]);
      vput(ebuf + (nxt * sg.e1_rows() + lr0 - 1) * nc, bp);
      const int wz = z + 1;
      if (own && wz >= 2 * K0 && wz < 2 * (K0 + KB))
        *reinterpret_cast<V*>(e1g + ((((wz & msk) << g.l2) + y) << (g.l2 - 1)) + m0) = bp;
    }
    // red residuals of plane z (RestrictCol's arithmetic), red values -r0/6
    if (z >= zs && rho_on) {
      const T* row = ebuf + (cur * sg.e1_rows() + lr0 - 1) * nc;
      const int par = (y + z) & 1;
      const V ow = *reinterpret_cast<const V*>(row + m0);
      const T edge = par ? row[(m0 + W) & cmsk] : row[(m0 - 1) & cmsk];
      const V vym = *reinterpret_cast<const V*>(row - nc + m0), vyp = *reinterpret_cast<const V*>(row + nc + m0);
      T rho[W];
#pragma unroll
      for (int q = 0; q < W; q++) {
        const T xm = par ? vget<T>(ow, q) : (q == 0 ? edge : vget<T>(ow, q - 1));
        const T xp = par ? (q == W - 1 ? edge : vget<T>(ow, q + 1)) : vget<T>(ow, q);
        const T nb = ((xm + xp) + (vget<T>(vym, q) + vget<T>(vyp, q))) + (vget<T>(bm, q) + vget<T>(bp, q));
        const T ev = neg_sixth(vget<T>(rz, q));
        rho[q] = vget<T>(rz, q) - (nb - T(6) * ev);
      }
      vput(hbuf + (lr0 - 2) * nc, make_float4(rho[0], rho[1], rho[2], rho[3]));
    }
    __syncthreads();
    if (z >= zs && coarse) {
      const int cz = z & 1;   // odd z = 2K + 1: last plane of K, first of K + 1
#pragma unroll
      for (int b = -1; b <= 1; b++) {
        const int yy = (2 * (J0 + Jl) + b) & msk;
        const int par = (yy + z) & 1;
        const T* rr = hbuf + (2 * Jl + b + 1) * nc;
        const V rv = *reinterpret_cast<const V*>(rr + m0);
        T row[W];
        if (par == 0) {
#pragma unroll
          for (int q = 0; q < W; q++) {
            T r = T(0);
            r += wt[1] * vget<T>(rv, q);
            row[q] = r;
          }
        } else {
          const T re = rr[(m0 - 1) & cmsk];
#pragma unroll
          for (int q = 0; q < W; q++) {
            T r = T(0);
            r += wt[0] * (q == 0 ? re : vget<T>(rv, q - 1));
            r += wt[2] * vget<T>(rv, q);
            row[q] = r;
          }
        }
        if (cz) {
          if (z > zs) {
            const T w = wt[b + 1] * wt[2];
#pragma unroll
            for (int q = 0; q < W; q++) sk[q] += w * row[q];
          }
          if (z < ze) {
            const T w = wt[b + 1] * wt[0];
#pragma unroll
            for (int q = 0; q < W; q++) sn[q] += w * row[q];
          }
        } else {
          const T w = wt[b + 1] * wt[1];
#pragma unroll
          for (int q = 0; q < W; q++) sk[q] += w * row[q];
        }
      }
      if (cz) {
        if (z > zs) {
          const int K = (z - 1) >> 1, J = J0 + Jl;
#pragma unroll
          for (int q = 0; q < W; q++) {
            const int I = m0 + q;
            T* out = ((I + J + K) & 1) ? A.rc1 : A.rc0;
            out[cs_index(gc, I, J, K)] = T(4) * sk[q];
          }
        }
#pragma unroll
        for (int q = 0; q < W; q++) {
          sk[q] = sn[q];
          sn[q] = T(0);
        }
      }
    }
    rz = rz1;
    rz1 = rz2;
    bm = bc;
    bc = bp;
    cur = nxt;
  }
}

// The up leg's two Gauss-Seidel sweeps after the black-only prolongation
// (red, black, red, black half-sweeps), FP32 on a 512^3 or 256^3 finest
// level of a single system, as one column walk instead of four launches:
// the input black values e1 are read once and the final red and black
// values written once (to s0 / s1: a workgroup reads its neighbours' input
// rows while they write their output, so the two must differ).  A workgroup
// owns JB fine rows (8 on 512^3, 16 on 256^3) of a band of KB planes; its
// JB + 8 thread rows are the owned rows with 4 more on each side, the y-halo
// the four dependent half-sweeps need (threads beyond them only join the
// barriers).
// At step k the first half-sweep updates plane k, the second plane k - 1,
// the third k - 2 and the fourth k - 3: each reads the previous half-sweep's
// plane in LDS (written one step before) for its x- and y-neighbours and
// its own row's neighbouring planes from registers.  Every value is formed
// with Halfsweep's arithmetic in its order, so the result is bitwise that of
// the four launches.  One workgroup barrier per step; LDS holds two buffers
// per half-sweep input.
constexpr int kPostThreads = 1024;
struct PostGeo {
  int nc, gx, JB, rows;   // JB owned fine rows per workgroup, rows = JB + 8 thread rows
  __host__ __device__ explicit PostGeo(int n) : nc(n / 2), gx(n / 8), JB(n >= 512 ? 8 : 16), rows(JB + 8) {}
  // LDS floats: two buffers of the inputs of the four half-sweeps (JB + 8, + 6, + 4, + 2 rows)
  __host__ __device__ int lds_floats() const { return 2 * (4 * JB + 20) * nc; }
};
struct PostSweeps {
  struct Args {
    int n;
    const float *e1, *r0, *r1;
    float *s0, *s1;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kPostThreads;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void PostSweeps::run(const Args& A, Grid G) {
  using T = float;
  using V = float4;
  constexpr int W = 4;
  if (A.ctl->done) return;
  const int n = A.n, msk = n - 1;
  const CsGeo g(n);
  const PostGeo pg(n);
  const int nc = pg.nc, gx = pg.gx, cmsk = nc - 1, JB = pg.JB;
  const int nj = n / JB, nz = G.g / nj, KB = n / nz;
  const int jb = G.b % nj, zr = G.b / nj;
  const int j0 = jb * JB, k0 = zr * KB;
  const int tid = threadIdx.x;
  const int r = tid / gx, m0 = (tid % gx) * W;   // thread row r: fine row j0 - 4 + r
  const int y = (j0 - 4 + r) & msk;
  const bool in0 = r < JB + 8;
  const bool in1 = r >= 1 && r < JB + 7, in2 = r >= 2 && r < JB + 6, in3 = r >= 3 && r < JB + 5;
  const bool in4 = r >= 4 && r < JB + 4;   // the workgroup's own rows
  extern __shared__ __align__(16) unsigned char ps_lds[];
  T* const L0 = reinterpret_cast<T*>(ps_lds);   // [2][16][nc] input black values
  T* const L1 = L0 + 2 * (JB + 8) * nc;         // [2][14][nc] first red
  T* const L2 = L1 + 2 * (JB + 6) * nc;         // [2][12][nc] first black
  T* const L3 = L2 + 2 * (JB + 4) * nc;         // [2][10][nc] second red
  auto at = [&](const T* a, int z) {
    return in0 ? *reinterpret_cast<const V*>(a + ((((z & msk) << g.l2) + y) << (g.l2 - 1)) + m0) : V{};
  };
  auto lds_row = [&](T* base, int nrows, int buf, int row) { return base + (buf * nrows + row) * nc; };
  // Halfsweep's update of W points of this row: neighbours of the other
  // colour from the LDS row (x and y) and the planes below / above (z)
  auto half = [&](const T* row, const V& zm, const V& zp, int par, const V& rc) {
    const V o = *reinterpret_cast<const V*>(row + m0);
    const T edge = par ? row[(m0 + W) & cmsk] : row[(m0 - 1) & cmsk];
    const V vym = *reinterpret_cast<const V*>(row - nc + m0), vyp = *reinterpret_cast<const V*>(row + nc + m0);
    T out[W];
#pragma unroll
    for (int q = 0; q < W; q++) {
      const T xm = par ? vget<T>(o, q) : (q == 0 ? edge : vget<T>(o, q - 1));
      const T xp = par ? (q == W - 1 ? edge : vget<T>(o, q + 1)) : vget<T>(o, q);
      const T nb = ((xm + xp) + (vget<T>(vym, q) + vget<T>(vyp, q))) + (vget<T>(zm, q) + vget<T>(zp, q));
      out[q] = (nb - vget<T>(rc, q)) * T(1.0 / 6.0);
    }
    return make_float4(out[0], out[1], out[2], out[3]);
  };
  auto put = [&](T* p, const V& v) { *reinterpret_cast<V*>(p + m0) = v; };
  const int kb = k0 - 3, ke = k0 + KB + 2;
  // register windows (this thread's row): input e of planes k-1, k, k+1;
  // first red at k-2, k-1; first black at k-3, k-2; second red at k-4, k-3;
  // r0 at k-1, k-2; r1 at k-2, k-3 (r0(k) and r1(k-1) arrive each step)
  V em = at(A.e1, kb - 1), ec = at(A.e1, kb), ep = at(A.e1, kb + 1), en = at(A.e1, kb + 2);
  V a1m{}, a1c{}, b2m{}, b2c{}, a3m{}, a3c{};
  V r0m = at(A.r0, kb - 1), r0mm = at(A.r0, kb - 2), r1m = at(A.r1, kb - 2), r1mm = at(A.r1, kb - 3);
  V r0n = at(A.r0, kb), r1n = at(A.r1, kb - 1);
  if (in0) put(lds_row(L0, JB + 8, 0, r), ec);
  __syncthreads();
  int cur = 0;
  for (int k = kb; k <= ke; k++) {
    const int nxt = cur ^ 1;
    const V r0k = r0n, r1k = r1n, e_next = en;   // r0(k), r1(k-1), e(k+2)
    if (k < ke) {
      en = at(A.e1, k + 3);
      r0n = at(A.r0, k + 1);
      r1n = at(A.r1, k);
    }
    V a1{}, b2{}, a3{};
    if (in1) {   // first red half-sweep, plane k
      a1 = half(lds_row(L0, JB + 8, cur, r), em, ep, (y + k) & 1, r0k);
      put(lds_row(L1, JB + 6, nxt, r - 1), a1);
    }
    if (in2) {   // first black half-sweep, plane k - 1
      b2 = half(lds_row(L1, JB + 6, cur, r - 1), a1m, a1, (1 + y + k - 1) & 1, r1k);
      put(lds_row(L2, JB + 4, nxt, r - 2), b2);
    }
    if (in3) {   // second red half-sweep, plane k - 2
      a3 = half(lds_row(L2, JB + 4, cur, r - 2), b2m, b2, (y + k - 2) & 1, r0mm);
      put(lds_row(L3, JB + 2, nxt, r - 3), a3);
      const int z = k - 2;
      if (in4 && z >= k0 && z < k0 + KB)
        *reinterpret_cast<V*>(A.s0 + ((((z & msk) << g.l2) + y) << (g.l2 - 1)) + m0) = a3;
    }
    if (in4) {   // second black half-sweep, plane k - 3
      const V b4 = half(lds_row(L3, JB + 2, cur, r - 3), a3m, a3, (1 + y + k - 3) & 1, r1mm);
      const int z = k - 3;
      if (z >= k0 && z < k0 + KB)
        *reinterpret_cast<V*>(A.s1 + ((((z & msk) << g.l2) + y) << (g.l2 - 1)) + m0) = b4;
    }
    if (in0) put(lds_row(L0, JB + 8, nxt, r), ep);   // the input's plane k + 1 for the next step
    __syncthreads();
    em = ec;
    ec = ep;
    ep = e_next;
    a1m = a1c;
    a1c = a1;
    b2m = b2c;
    b2c = b2;
    a3m = a3c;
    a3c = a3;
    r0mm = r0m;
    r0m = r0k;
    r1mm = r1m;
    r1m = r1k;
    cur = nxt;
  }
}

// Trilinear interpolation of the coarse correction (colour-split, geometry
// gc) at fine point (x,y,z).
template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ c0, const T* __restrict__ c1, const CsGeo& gc, int x,
                                        int y, int z) {
  const int cm = gc.n - 1;
  const int x0 = x >> 1, y0 = y >> 1, z0 = z >> 1;
  const int x1 = (x & 1) ? ((x0 + 1) & cm) : x0;
  const int y1 = (y & 1) ? ((y0 + 1) & cm) : y0;
  const int z1 = (z & 1) ? ((z0 + 1) & cm) : z0;
  const T hx = (x & 1) ? T(0.5) : T(1), hy = (y & 1) ? T(0.5) : T(1), hz = (z & 1) ? T(0.5) : T(1);
  T s = T(0);
  const int xs[2] = {x0, x1}, ys[2] = {y0, y1}, zs[2] = {z0, z1};
  const int nx = (x & 1) ? 2 : 1, ny = (y & 1) ? 2 : 1, nz = (z & 1) ? 2 : 1;
  for (int c = 0; c < nz; c++)
    for (int b = 0; b < ny; b++)
      for (int a = 0; a < nx; a++) {
        const T* arr = ((xs[a] + ys[b] + zs[c]) & 1) ? c1 : c0;
        s += hx * hy * hz * arr[cs_index(gc, xs[a], ys[b], zs[c])];
      }
  return s;
}

// Black points x = 2m + sx, m = m0 .. m0+W-1, of the row (j,k) holding the
// colour-split index t, plus their trilinear coarse correction: weights and
// coarse indices as in prolong_at, summed in its order with exact zeros
// interleaved (so the values equal e1[t+q] + prolong_at(...) exactly); the
// coarse values of each coarse row are loaded once for the W points.
template <typename T>
__device__ __forceinline__ typename Vec<T>::type prolong_black_vec(const T* e1, const T* ec0, const T* ec1,
                                                                  const CsGeo& g, const CsGeo& gc, int t) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  int m0, j, k;
  cs_decode(g, t, &m0, &j, &k);
  const int sx = (1 + j + k) & 1, cm = gc.n - 1;
  const int y0 = j >> 1, z0 = k >> 1;
  const int ys[2] = {y0, (j & 1) ? ((y0 + 1) & cm) : y0};
  const int zs[2] = {z0, (k & 1) ? ((z0 + 1) & cm) : z0};
  const T hx = sx ? T(0.5) : T(1), hy = (j & 1) ? T(0.5) : T(1), hz = (k & 1) ? T(0.5) : T(1);
  // a coarse row that an even fine index does not use (second y or z entry)
  // gets weight 0: it adds exact zeros, so all four rows can be loaded at once
  const T wy[2] = {hy, (j & 1) ? hy : T(0)}, wz[2] = {hz, (k & 1) ? hz : T(0)};
  const T wx1 = sx ? T(1) : T(0);
  T acc[W];
#pragma unroll
  for (int q = 0; q < W; q++) acc[q] = T(0);
#pragma unroll
  for (int c = 0; c < 2; c++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int Y = ys[b], Z = zs[c];
      const int crow = ((Z << gc.l2) + Y) << (gc.l2 - 1);
      const T w = hx * wy[b] * wz[c];
      T cv[W + 1];   // coarse values at X = m0 .. m0+W (wrapped)
#pragma unroll
      for (int q = 0; q <= W; q++) {
        const int X = (m0 + q) & cm;
        cv[q] = (((X + Y + Z) & 1) ? ec1 : ec0)[crow + (X >> 1)];
      }
#pragma unroll
      for (int q = 0; q < W; q++) {
        acc[q] += w * cv[q];
        acc[q] += (w * wx1) * cv[q + 1];
      }
    }
  const V old = *reinterpret_cast<const V*>(e1 + t);
  V out;
#pragma unroll
  for (int q = 0; q < W; q++) vset<T>(out, q, vget<T>(old, q) + acc[q]);
  return out;
}

// After prolongation the next red half-sweep overwrites every red value and
// reads only black neighbours, so only the black points receive the
// trilinear correction here; the red half-sweep follows.
template <typename T, int FIN, int SPEC>
struct ProlongBlack {
  struct Args {
    int n;
    T* e1;
    const T *ec0, *ec1;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN, int SPEC>
__device__ void ProlongBlack<T, FIN, SPEC>::run(const Args& A, Grid G) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const int n = A.n;
  T* __restrict__ e1 = A.e1;
  const T* __restrict__ ec0 = A.ec0;
  const T* __restrict__ ec1 = A.ec1;
  const int done = A.ctl->done;
  if (!SPEC && done) return;
  const CsGeo g(n), gc(n >> 1);
  const int half = n * g.hn * n;
  const int t = (G.b * kBlock + threadIdx.x) * W;
  if (t >= half) return;
  const V out = prolong_black_vec(e1, ec0, ec1, g, gc, t);
  if (SPEC) {
    keep_issued(out);
    if (done) return;
  }
  *reinterpret_cast<V*>(e1 + t) = out;
}

// ProlongBlack from 256^3 up: each thread walks kProlongPlanes fine z-planes
// of its W black points, keeping the coarse rows of the two coarse planes it
// interpolates between in registers, so each coarse row is loaded once per
// two fine planes instead of four times per plane.  Per point the terms are
// those of prolong_black_vec in the same order (the same rows, weights and
// exact zeros), so the result is bitwise the same.
constexpr int kProlongPlanes = 16;
template <typename T, int FIN>
struct ProlongCol {
  using Args = typename ProlongBlack<T, FIN, 0>::Args;
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int FIN>
__device__ void ProlongCol<T, FIN>::run(const Args& A, Grid G) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  if (A.ctl->done) return;
  const int n = A.n;
  T* __restrict__ e1 = A.e1;
  const T* __restrict__ ec0 = A.ec0;
  const T* __restrict__ ec1 = A.ec1;
  const CsGeo g(n), gc(n >> 1);
  const int per_plane = g.plane / W;                  // threads of one fine plane
  const int tp = (G.b * kBlock + threadIdx.x);
  const int band = tp / per_plane, u = tp % per_plane;
  const int m0 = (u * W) & (g.hn - 1), j = (u * W) >> (g.l2 - 1);
  const int k0 = band * kProlongPlanes;
  if (k0 >= n) return;
  const int cm = gc.n - 1, y0 = j >> 1;
  const int ys[2] = {y0, (j & 1) ? ((y0 + 1) & cm) : y0};
  const T hy = (j & 1) ? T(0.5) : T(1);
  const T wy[2] = {hy, (j & 1) ? hy : T(0)};
  // coarse values at X = m0 .. m0 + W of rows ys[0], ys[1] of coarse plane Z
  auto load_plane = [&](int Z, T (*cv)[W + 1]) {
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int Y = ys[b];
      const int crow = ((Z << gc.l2) + Y) << (gc.l2 - 1);
#pragma unroll
      for (int q = 0; q <= W; q++) {
        const int X = (m0 + q) & cm;
        cv[b][q] = (((X + Y + Z) & 1) ? ec1 : ec0)[crow + (X >> 1)];
      }
    }
  };
  T lo[2][W + 1], hi[2][W + 1];   // coarse planes k >> 1 and (k >> 1) + 1
  load_plane((k0 >> 1) & cm, lo);
  for (int kk = 0; kk < kProlongPlanes; kk++) {
    const int k = k0 + kk;
    if ((k & 1) == 0) {
      if (kk > 0) {
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
          for (int q = 0; q <= W; q++) lo[b][q] = hi[b][q];
      }
      load_plane(((k >> 1) + 1) & cm, hi);
    } else if (kk == 0) {
      load_plane(((k >> 1) + 1) & cm, hi);
    }
    const int t = ((k << g.l2) + j) * g.hn + m0;
    const int sx = (1 + j + k) & 1;
    const T hx = sx ? T(0.5) : T(1), hz = (k & 1) ? T(0.5) : T(1);
    const T wz[2] = {hz, (k & 1) ? hz : T(0)};
    const T wx1 = sx ? T(1) : T(0);
    T acc[W];
#pragma unroll
    for (int q = 0; q < W; q++) acc[q] = T(0);
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
      for (int b = 0; b < 2; b++) {
        // the second z entry of an even fine plane is the first coarse plane again (weight 0)
        const T* cv = (c == 1 && (k & 1)) ? hi[b] : lo[b];
        const T w = hx * wy[b] * wz[c];
#pragma unroll
        for (int q = 0; q < W; q++) {
          acc[q] += w * cv[q];
          acc[q] += (w * wx1) * cv[q + 1];
        }
      }
    const V old = *reinterpret_cast<const V*>(e1 + t);
    V out;
#pragma unroll
    for (int q = 0; q < W; q++) vset<T>(out, q, vget<T>(old, q) + acc[q]);
    *reinterpret_cast<V*>(e1 + t) = out;
  }
}

template <typename T>
struct ProlongAdd {
  struct Args {
    int n;
    T *e0, *e1;
    const T *ec0, *ec1;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T>
__device__ void ProlongAdd<T>::run(const Args& A, Grid G) {
  const int n = A.n;
  T* __restrict__ e0 = A.e0;
  T* __restrict__ e1 = A.e1;
  const T* __restrict__ ec0 = A.ec0;
  const T* __restrict__ ec1 = A.ec1;
  if (A.ctl->done) return;
  const CsGeo g(n), gc(n >> 1);
  const int half = n * g.hn * n;
  const int t = G.b * kBlock + threadIdx.x;
  if (t >= half) return;
  int m, j, k;
  cs_decode(g, t, &m, &j, &k);
  const int ir = 2 * m + ((j + k) & 1), ib = 2 * m + ((1 + j + k) & 1);
  e0[t] += prolong_at(ec0, ec1, gc, ir, j, k);
  e1[t] += prolong_at(ec0, ec1, gc, ib, j, k);
}

template <typename T>
struct FillZero {
  struct Args {
    int64_t count;
    T *a, *b;
    const Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    if (A.ctl->done) return;
    const int64_t t = (int64_t)G.b * kBlock + threadIdx.x;
    if (t < A.count) {
      A.a[t] = T(0);
      A.b[t] = T(0);
    }
  }
};

// ---------------------------------------------------------------------------
// Fused smoothing of a small level (temporal blocking).  On levels whose
// kernels are bound by launch and memory latency rather than bandwidth, one
// launch runs a whole leg's chain of half-sweeps: a workgroup owns a tile of
// TY x TZ full x-rows and holds, in LDS, a box of rows around it with a halo
// of S rows in y and z (S = number of neighbour-dependent half-sweeps).  The
// first operation is pointwise and fills the box; half-sweep s then updates
// the box shrunk to halo S-1-s, so the last one produces the tile itself.
// Every point value is computed with the arithmetic, operand order and
// neighbour order of the unfused kernels (SweepZero, ProlongBlack,
// Halfsweep), so the level's result is bitwise that of the unfused chain;
// halo values are recomputed redundantly by neighbouring tiles.
//   down leg (UP = 0): red = -r/6 everywhere (first sweep from e = 0), then
//     black, red, ... (S = 2 nu1 - 1 half-sweeps); out = down-leg buffers.
//   up leg (UP = 1): black += trilinear correction (ProlongBlack), then red,
//     black, ... (S = 2 nu2 half-sweeps).  The black input (the down leg's
//     result) and the output are different buffers: a tile reads its halo
//     rows while neighbouring tiles write their own rows.
// LDS: e of both colours on the box (halo S), r of both colours on the box
// shrunk by one (halo S-1), rows of n/2 elements per colour.
// ---------------------------------------------------------------------------
struct FusedBox {
  int by, bz, ry, rz;   // rows of the e box (halo S + hb) and of the r box (one less)
  size_t elems;         // LDS elements of e0, e1, r0, r1
  FusedBox(int n, int ty, int tz, int S, int hb)
      : by(ty + 2 * (S + hb)), bz(tz + 2 * (S + hb)), ry(by - 2), rz(bz - 2),
        elems((size_t)(n / 2) * (2 * (size_t)by * bz + 2 * (size_t)ry * rz)) {}
};

// RST (down leg only): the launch also forms the restricted red residual of
// its tile's coarse points (RestrictRed's arithmetic, in its order) into the
// coarse right-hand side rc0/rc1.  That needs the final black values two rows
// and the final red values one row around the tile, so every half-sweep runs
// on a box two rows wider (hb = 2).
template <typename T, int UP, int FIN, int RST>
struct Fused {
  struct Args {
    int n, ty, tz, steps;
    const T *r0, *r1;
    const T* src1;          // up leg: black values of the down leg
    const T *ec0, *ec1;     // up leg: coarse correction (colour-split, edge n/2)
    T *out0, *out1;
    T *rc0, *rc1;           // RST: coarse right-hand side (colour-split, edge n/2)
    const Ctl* ctl;
  };
  // one workgroup per compute unit on a 64^3 level: every phase of the
  // halo box is one pass of the workgroup, so the global loads of the first
  // operation are issued at once
  static constexpr int kThreads = 1024;
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, int UP, int FIN, int RST>
__device__ void Fused<T, UP, FIN, RST>::run(const Args& A, Grid G) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  constexpr int HB = RST ? 2 : 0;
  const int done = A.ctl->done;
  const int n = A.n, hn = n >> 1, msk = n - 1, S = A.steps, TY = A.ty, TZ = A.tz;
  const int SB = S + HB;   // halo of the e box
  const int BY = TY + 2 * SB, BZ = TZ + 2 * SB, RY = BY - 2, RZ = BZ - 2;
  const int nty = n / TY;
  const int y0 = (G.b % nty) * TY, z0 = (G.b / nty) * TZ;
  const int vl2 = __builtin_ctz(hn / W), vmsk = hn / W - 1;   // vectors per colour row
  extern __shared__ __align__(16) unsigned char fused_lds[];
  T* const E0 = reinterpret_cast<T*>(fused_lds);
  T* const E1 = E0 + (size_t)BY * BZ * hn;
  T* const R0 = E1 + (size_t)BY * BZ * hn;
  T* const R1 = R0 + (size_t)RY * RZ * hn;
  const int tid = threadIdx.x, nt = blockDim.x;
  const CsGeo g(n), gc(n >> 1);
  const T sixth = T(1.0 / 6.0);
  // pointwise first operation on the whole box; r of both colours into the
  // inner box
  const int cinit = UP ? 1 : 0;
  T* const Ei = UP ? E1 : E0;
  for (int task = tid; task < BY * BZ * (hn / W); task += nt) {
    const int row = task >> vl2, m = (task & vmsk) * W;
    const int ey = row % BY, ez = row / BY;   // box coordinates
    const int j = (y0 + ey - SB) & msk, k = (z0 + ez - SB) & msk;
    const int t = ((k << g.l2) + j) * hn + m;
    V v;
    if (UP) {
      v = prolong_black_vec(A.src1, A.ec0, A.ec1, g, gc, t);
    } else {
      const V rr = *reinterpret_cast<const V*>(A.r0 + t);
#pragma unroll
      for (int q = 0; q < W; q++) vset<T>(v, q, neg_sixth(vget<T>(rr, q)));
    }
    *reinterpret_cast<V*>(Ei + row * hn + m) = v;
    if (ey >= 1 && ey <= RY && ez >= 1 && ez <= RZ) {
      const int rrow = (ez - 1) * RY + (ey - 1);
      *reinterpret_cast<V*>(R0 + rrow * hn + m) = *reinterpret_cast<const V*>(A.r0 + t);
      *reinterpret_cast<V*>(R1 + rrow * hn + m) = *reinterpret_cast<const V*>(A.r1 + t);
    }
  }
  if (done) return;   // uniform: nothing has been written to global memory
  __syncthreads();
  for (int st = 0; st < S; st++) {
    const int c = (cinit + 1 + st) & 1, h = S - 1 - st + HB;   // colour and halo of this half-sweep
    const int HY = TY + 2 * h, HZ = TZ + 2 * h;
    T* const Ec = c ? E1 : E0;
    const T* const Eo = c ? E0 : E1;
    const T* const Rc = c ? R1 : R0;
    const bool out_now = !RST && st == S - 1;   // the last half-sweep writes the tile to global memory
    for (int task = tid; task < HY * HZ * (hn / W); task += nt) {
      const int hrow = task >> vl2, m = (task & vmsk) * W;
      const int dy = hrow % HY + (SB - h), dz = hrow / HY + (SB - h);   // box coordinates
      const int j = (y0 + dy - SB) & msk, k = (z0 + dz - SB) & msk;
      const int row = dz * BY + dy;
      const int sp = (c + j + k) & 1;   // x-parity of this colour in the row
      const T* o = Eo + row * hn;
      const V own = *reinterpret_cast<const V*>(o + m);
      const T edge = sp ? o[m + W == hn ? 0 : m + W] : o[m == 0 ? hn - 1 : m - 1];
      const V vym = *reinterpret_cast<const V*>(o - hn + m), vyp = *reinterpret_cast<const V*>(o + hn + m);
      const V vzm = *reinterpret_cast<const V*>(o - BY * hn + m), vzp = *reinterpret_cast<const V*>(o + BY * hn + m);
      const V rv = *reinterpret_cast<const V*>(Rc + ((dz - 1) * RY + (dy - 1)) * hn + m);
      V out;
#pragma unroll
      for (int q = 0; q < W; q++) {
        const T xm = sp ? vget<T>(own, q) : (q == 0 ? edge : vget<T>(own, q - 1));
        const T xp = sp ? (q == W - 1 ? edge : vget<T>(own, q + 1)) : vget<T>(own, q);
        const T nb = ((xm + xp) + (vget<T>(vym, q) + vget<T>(vyp, q))) + (vget<T>(vzm, q) + vget<T>(vzp, q));
        vset<T>(out, q, (nb - vget<T>(rv, q)) * sixth);
      }
      if (out_now) {
        // the tile: this colour from the last half-sweep, the other colour
        // from the one before (or the first operation)
        const int t = ((k << g.l2) + j) * hn + m;
        *reinterpret_cast<V*>((c ? A.out1 : A.out0) + t) = out;
        *reinterpret_cast<V*>((c ? A.out0 : A.out1) + t) = own;
      } else {
        *reinterpret_cast<V*>(Ec + row * hn + m) = out;
      }
    }
    if (!out_now) __syncthreads();
  }
  if (!RST) return;
  // the tile's rows of both colours
  for (int task = tid; task < TY * TZ * (hn / W); task += nt) {
    const int trow = task >> vl2, m = (task & vmsk) * W;
    const int dy = trow % TY + SB, dz = trow / TY + SB;
    const int j = (y0 + dy - SB) & msk, k = (z0 + dz - SB) & msk;
    const int row = dz * BY + dy;
    const int t = ((k << g.l2) + j) * hn + m;
    *reinterpret_cast<V*>(A.out0 + t) = *reinterpret_cast<const V*>(E0 + row * hn + m);
    *reinterpret_cast<V*>(A.out1 + t) = *reinterpret_cast<const V*>(E1 + row * hn + m);
  }
  // restricted red residual at the tile's coarse points: coarse rows
  // J = y0/2 .. (y0+TY)/2 - 1 (likewise K), W coarse points per task
  const int cty = TY >> 1, ctz = TZ >> 1, nc = hn, cvl2 = __builtin_ctz(nc / W);
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  for (int task = tid; task < cty * ctz * (nc / W); task += nt) {
    const int crow = task >> cvl2, I0 = (task & (nc / W - 1)) * W;
    const int J = (y0 >> 1) + crow % cty, K = (z0 >> 1) + crow / cty;
    T sacc[W];
#pragma unroll
    for (int q = 0; q < W; q++) sacc[q] = T(0);
    // three rows at a time (all nine unrolled spill)
#pragma unroll 1
    for (int cz = -1; cz <= 1; cz++) {
      const int dz = 2 * K + cz - z0 + SB;   // box row of fine z = 2K + cz
      const int z = (2 * K + cz) & msk;
#pragma unroll
      for (int by = -1; by <= 1; by++) {
        const int dy = 2 * J + by - y0 + SB;
        const int y = (2 * J + by) & msk;
        const int par = (y + z) & 1;   // red points of this row sit at x = 2m + par
        const int row = dz * BY + dy;
        const T* o = E1 + row * hn;
        const V own = *reinterpret_cast<const V*>(o + I0);
        const T edge = par ? o[I0 + W == hn ? 0 : I0 + W] : o[I0 == 0 ? hn - 1 : I0 - 1];
        const V vym = *reinterpret_cast<const V*>(o - hn + I0), vyp = *reinterpret_cast<const V*>(o + hn + I0);
        const V vzm = *reinterpret_cast<const V*>(o - BY * hn + I0), vzp = *reinterpret_cast<const V*>(o + BY * hn + I0);
        const V ev = *reinterpret_cast<const V*>(E0 + row * hn + I0);
        const T* rr = R0 + ((dz - 1) * RY + (dy - 1)) * hn;
        const V rv = *reinterpret_cast<const V*>(rr + I0);
        T rho[W];
#pragma unroll
        for (int q = 0; q < W; q++) {
          const T xm = par ? vget<T>(own, q) : (q == 0 ? edge : vget<T>(own, q - 1));
          const T xp = par ? (q == W - 1 ? edge : vget<T>(own, q + 1)) : vget<T>(own, q);
          const T nb = ((xm + xp) + (vget<T>(vym, q) + vget<T>(vyp, q))) + (vget<T>(vzm, q) + vget<T>(vzp, q));
          rho[q] = vget<T>(rv, q) - (nb - T(6) * vget<T>(ev, q));
        }
        const T wbc = wt[by + 1] * wt[cz + 1];
        if (par == 0) {
          // only x = 2I is red: m = I
#pragma unroll
          for (int q = 0; q < W; q++) {
            T rowsum = T(0);
            rowsum += wt[1] * rho[q];
            sacc[q] += wbc * rowsum;
          }
        } else {
          // x = 2I - 1 (m = I - 1) and x = 2I + 1 (m = I)
          const int me = (I0 - 1) & (hn - 1);
          const T xm = o[me], xp = o[me + 1 == hn ? 0 : me + 1];
          const T nbe = ((xm + xp) + (o[me - hn] + o[me + hn])) + (o[me - BY * hn] + o[me + BY * hn]);
          const T rho_e = rr[me] - (nbe - T(6) * E0[row * hn + me]);
#pragma unroll
          for (int q = 0; q < W; q++) {
            T rowsum = T(0);
            rowsum += wt[0] * (q == 0 ? rho_e : rho[q - 1]);
            rowsum += wt[2] * rho[q];
            sacc[q] += wbc * rowsum;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < W; q++) {
      const int I = I0 + q;
      (((I + J + K) & 1) ? A.rc1 : A.rc0)[cs_index(gc, I, J, K)] = T(4) * sacc[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Tail of the V-cycle: all levels from n0 down to 4^3 and back in one
// workgroup, with the exact coarsest solve e = G * r (G the periodic 4^3
// Green's function of M, FP64 accumulation).  Levels up to 16^3 are
// LDS-resident in the same colour-split layout as the upper levels; a top
// level of 32^3 (batched systems) stays in global memory.  Each phase
// performs the operation of the corresponding multi-workgroup kernel above
// with the same order of operations, so a level's result does not depend on
// where it runs; sweeps, the first sweep from zero and the residual work on
// 16-byte row vectors.  LDS per level q (edge n_q): e0, e1, r0, r1 of
// n_q^3/2 elements each, then the red residuals of the current level.
// ---------------------------------------------------------------------------
// Full weighting x 4 at the coarse points I0 .. I0+W-1 of coarse row (J,K)
// from the red residuals rho (red colour array of the fine level; the black
// residuals are zero), with the terms and their order of ResidRestrict.
template <typename T>
__device__ __forceinline__ void restrict_red_vec(const T* rho, const CsGeo& g, int I0, int J, int K, T* v) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  const int msk = g.n - 1, hm = g.hn - 1;
  T s[W];
#pragma unroll
  for (int q = 0; q < W; q++) s[q] = T(0);
#pragma unroll
  for (int c = -1; c <= 1; c++) {
    const int z = (2 * K + c) & msk;
#pragma unroll
    for (int b = -1; b <= 1; b++) {
      const int y = (2 * J + b) & msk;
      const int row0 = ((z << g.l2) + y) << (g.l2 - 1);
      const V rv = *reinterpret_cast<const V*>(rho + row0 + I0);
      const T wbc = wt[b + 1] * wt[c + 1];
      if (((b + c) & 1) == 0) {
#pragma unroll
        for (int q = 0; q < W; q++) {
          T row = T(0);
          row += wt[1] * vget<T>(rv, q);
          s[q] += wbc * row;
        }
      } else {
        const T re = rho[row0 + ((I0 - 1) & hm)];
#pragma unroll
        for (int q = 0; q < W; q++) {
          T row = T(0);
          row += wt[0] * (q == 0 ? re : vget<T>(rv, q - 1));
          row += wt[2] * vget<T>(rv, q);
          s[q] += wbc * row;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < W; q++) v[q] = T(4) * s[q];
}

__device__ __forceinline__ int tail_level_offset(int n0, int q) {
  int off = 0;
  for (int p = 0; p < q; p++) {
    const int n = n0 >> p;
    off += 2 * n * n * n;
  }
  return off;
}

// One half-sweep of colour `colour` (Halfsweep on LDS or global arrays).
template <typename T>
__device__ __forceinline__ void tail_half(T* ec, const T* eo, const T* rc, const CsGeo& g, int half, int colour) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  for (int t = threadIdx.x * W; t < half; t += blockDim.x * W) {
    int m, j, k;
    cs_decode(g, t, &m, &j, &k);
    T nb[W];
    cs_nbr6_vec(eo, g, t, m, j, k, (colour + j + k) & 1, [](T x) { return x; }, nb);
    const V r = *reinterpret_cast<const V*>(rc + t);
    V out;
#pragma unroll
    for (int q = 0; q < W; q++) vset<T>(out, q, (nb[q] - vget<T>(r, q)) * T(1.0 / 6.0));
    *reinterpret_cast<V*>(ec + t) = out;
  }
}

// Levels of the tail up to this edge live in LDS; a tail whose top level is
// larger keeps that one level in global memory (same workgroup, so its
// phases are ordered by the same barriers) and the rest in LDS.
constexpr int kTailLdsMax = 16;

template <typename T>
struct Tail {
  struct Args {
    int n0, levels, nu1, nu2;
    const T *r0, *r1;
    T *e0, *e1;
    const double* green;
    Ctl* ctl;
    // the pending stop decision of the previous outer residual (partial
    // null: none is made here)
    const double* partial;
    int nb, n3, max_cycles;
  };
  static constexpr int kThreads = 1024;
  __device__ static void run(const Args& A, Grid G);
};
// One level of the descending leg on level arrays of edge n (the pointers
// may be global or LDS; the functions are inlined per call site so each
// access keeps its own address space): nu1 sweeps, the first from e = 0,
// then the restricted residual into the next level's right-hand side rc.
// GL: a level in global memory forms the red residuals inside the
// restriction (RestrictRed); an LDS level writes them to rho first
// (ResidRestrict).
template <typename T, bool GL>
__device__ __forceinline__ void tail_down(T* e0, T* e1, const T* r0, const T* r1, T* rc0, T* rc1, T* rho, int n,
                                          int nu1) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int half = n * n * n / 2;
  const CsGeo g(n);
  const int nc = n >> 1;
  const CsGeo gc(nc);
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  if (nu1 >= 1) {
    // first sweep from e = 0 (SweepZero): red = -r/6, black from those reds
    const T sixth = T(1.0 / 6.0);
    for (int t = tid * W; t < half; t += nt * W) {
      int m, j, k;
      cs_decode(g, t, &m, &j, &k);
      const V rr = *reinterpret_cast<const V*>(r0 + t);
      V er;
#pragma unroll
      for (int c = 0; c < W; c++) vset<T>(er, c, neg_sixth(vget<T>(rr, c)));
      *reinterpret_cast<V*>(e0 + t) = er;
      T nb[W];
      cs_nbr6_vec(r0, g, t, m, j, k, (1 + j + k) & 1, [](T x) { return neg_sixth(x); }, nb);
      const V rb = *reinterpret_cast<const V*>(r1 + t);
      V eb;
#pragma unroll
      for (int c = 0; c < W; c++) vset<T>(eb, c, (nb[c] - vget<T>(rb, c)) * sixth);
      *reinterpret_cast<V*>(e1 + t) = eb;
    }
    __syncthreads();
    for (int it = 1; it < nu1; it++) {
      tail_half(e0, e1, r0, g, half, 0);
      __syncthreads();
      tail_half(e1, e0, r1, g, half, 1);
      __syncthreads();
    }
    if (GL) {
      for (int p = tid * W; p < nc * nc * nc; p += nt * W) {
        const int I0 = p & (nc - 1), J = (p >> gc.l2) & (nc - 1), K = p >> (2 * gc.l2);
        T v[W];
        restrict_red_recompute<T, 1>(e0, e1, r0, g, I0, J, K, v);
#pragma unroll
        for (int c = 0; c < W; c++) {
          const int I = I0 + c;
          (((I + J + K) & 1) ? rc1 : rc0)[cs_index(gc, I, J, K)] = v[c];
        }
      }
      __syncthreads();
      return;
    }
    // residual at the red points; after the black half-sweep the black
    // residuals vanish up to rounding and are taken as zero
    for (int t = tid * W; t < half; t += nt * W) {
      int m, j, k;
      cs_decode(g, t, &m, &j, &k);
      T nb[W];
      cs_nbr6_vec(e1, g, t, m, j, k, (j + k) & 1, [](T x) { return x; }, nb);
      const V ev = *reinterpret_cast<const V*>(e0 + t);
      const V rv = *reinterpret_cast<const V*>(r0 + t);
      V out;
#pragma unroll
      for (int c = 0; c < W; c++) vset<T>(out, c, vget<T>(rv, c) - (nb[c] - T(6) * vget<T>(ev, c)));
      *reinterpret_cast<V*>(rho + t) = out;
    }
    __syncthreads();
    // full weighting x 4 into the next level's right-hand side
    for (int p = tid * W; p < nc * nc * nc; p += nt * W) {
      const int I0 = p & (nc - 1), J = (p >> gc.l2) & (nc - 1), K = p >> (2 * gc.l2);
      T v[W];
      restrict_red_vec(rho, g, I0, J, K, v);
#pragma unroll
      for (int c = 0; c < W; c++) {
        const int I = I0 + c;
        (((I + J + K) & 1) ? rc1 : rc0)[cs_index(gc, I, J, K)] = v[c];
      }
    }
    __syncthreads();
    return;
  }
  // no pre-smoothing: e = 0 and the residual is r itself at every point
  for (int t = tid; t < half; t += nt) {
    e0[t] = T(0);
    e1[t] = T(0);
  }
  __syncthreads();
  const int msk = n - 1;
  for (int p = tid; p < nc * nc * nc; p += nt) {
    const int I = p & (nc - 1), J = (p >> gc.l2) & (nc - 1), K = p >> (2 * gc.l2);
    T s = T(0);
    for (int c = -1; c <= 1; c++) {
      const int z = (2 * K + c) & msk;
      for (int b = -1; b <= 1; b++) {
        const int y = (2 * J + b) & msk;
        T row = T(0);
        for (int a = -1; a <= 1; a++) {
          const int x = (2 * I + a) & msk;
          const int odd = (x + y + z) & 1;
          const int ti = cs_index(g, x, y, z);
          row += wt[a + 1] * (odd ? r1[ti] : r0[ti]);
        }
        s += wt[b + 1] * wt[c + 1] * row;
      }
    }
    T* out = ((I + J + K) & 1) ? rc1 : rc0;
    out[cs_index(gc, I, J, K)] = T(4) * s;
  }
  __syncthreads();
}

// One level of the ascending leg: trilinear correction from the coarse
// level (c0, c1), then nu2 sweeps.
template <typename T>
__device__ __forceinline__ void tail_up(T* e0, T* e1, const T* r0, const T* r1, const T* c0, const T* c1, int n,
                                        int nu2) {
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int half = n * n * n / 2;
  const CsGeo g(n), gc(n >> 1);
  if (nu2 >= 1) {
    // the next red half-sweep overwrites every red point: only black points
    // take the correction (ProlongBlack)
    for (int t = tid * W; t < half; t += nt * W)
      *reinterpret_cast<V*>(e1 + t) = prolong_black_vec(e1, c0, c1, g, gc, t);
    __syncthreads();
    for (int it = 0; it < nu2; it++) {
      tail_half(e0, e1, r0, g, half, 0);
      __syncthreads();
      tail_half(e1, e0, r1, g, half, 1);
      __syncthreads();
    }
  } else {
    for (int t = tid; t < half; t += nt) {
      int m, j, k;
      cs_decode(g, t, &m, &j, &k);
      e0[t] += prolong_at(c0, c1, gc, 2 * m + ((j + k) & 1), j, k);
      e1[t] += prolong_at(c0, c1, gc, 2 * m + ((1 + j + k) & 1), j, k);
    }
    __syncthreads();
  }
}

// GTOP: the top level (edge n0 > kTailLdsMax) stays in global memory and
// the LDS holds the levels below it.
template <typename T, bool GTOP>
__device__ __forceinline__ void tail_run(const typename Tail<T>::Args& A, int done) {
  // (done: the control block's flag, replaced by the pending stop decision
  // when this launch makes it)
  const int n0 = A.n0, levels = A.levels, nu1 = A.nu1, nu2 = A.nu2;
  constexpr int W = Vec<T>::W;
  using V = typename Vec<T>::type;
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ double G[64];
  T* const base = reinterpret_cast<T*>(tail_lds);
  // LDS level q has edge nl >> q
  const int nl = GTOP ? n0 >> 1 : n0, ll = GTOP ? levels - 1 : levels;
  T* const rho = base + tail_level_offset(nl, ll);   // red residuals of an LDS level
  auto E0 = [&](int q) -> T* { return base + tail_level_offset(nl, q); };
  auto E1 = [&](int q) -> T* {
    const int n = nl >> q;
    return E0(q) + n * n * n / 2;
  };
  auto R0 = [&](int q) -> T* {
    const int n = nl >> q;
    return E0(q) + n * n * n;
  };
  auto R1 = [&](int q) -> T* {
    const int n = nl >> q;
    return E0(q) + 3 * (n * n * n / 2);
  };
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid < 64) G[tid] = A.green[tid];
  if (!GTOP) {
    // the top level is in LDS: its right-hand side comes from global memory
    const int half = n0 * n0 * n0 / 2;
    T* r0 = R0(0);
    T* r1 = R1(0);
    for (int t = tid; t < half; t += nt) {
      r0[t] = A.r0[t];
      r1[t] = A.r1[t];
    }
  }
  if (A.partial) {
    // the pending stop decision, its partials loaded alongside the level data
    __shared__ double sh[32];
    __shared__ DecideOut out;
    outer_decide(A.ctl, A.partial, A.nb, A.n3, A.max_cycles, true, true, sh, &out);
    done = out.done;
  }
  if (done) return;
  __syncthreads();
  if (GTOP) tail_down<T, true>(A.e0, A.e1, A.r0, A.r1, R0(0), R1(0), rho, n0, nu1);
  for (int q = 0; q + 1 < ll; q++)
    tail_down<T, false>(E0(q), E1(q), R0(q), R1(q), R0(q + 1), R1(q + 1), rho, nl >> q, nu1);
  {
    // 4^3: e = G * r with FP64 accumulation; 16 consecutive lanes share one
    // output point, each summing 4 of the 64 terms, then a fixed shuffle tree
    const int q = ll - 1;
    T* e0 = E0(q);
    T* e1 = E1(q);
    const T* r0 = R0(q);
    const T* r1 = R1(q);
    const CsGeo g4(4);
    const int o = tid >> 4, part = tid & 15;
    double s = 0.0;
    if (o < 64) {
      const int x = o & 3, y = (o >> 2) & 3, z = o >> 4;
      for (int mm = part * 4; mm < part * 4 + 4; mm++) {
        const int a = mm & 3, b = (mm >> 2) & 3, c = mm >> 4;
        const T rv = ((a + b + c) & 1) ? r1[cs_index(g4, a, b, c)] : r0[cs_index(g4, a, b, c)];
        s += G[(((z - c) & 3) * 4 + ((y - b) & 3)) * 4 + ((x - a) & 3)] * (double)rv;
      }
    }
    for (int d = 8; d > 0; d >>= 1) s += __shfl_xor(s, d, 16);
    if (o < 64 && part == 0) {
      const int x = o & 3, y = (o >> 2) & 3, z = o >> 4;
      (((x + y + z) & 1) ? e1 : e0)[cs_index(g4, x, y, z)] = (T)s;
    }
    __syncthreads();
  }
  for (int q = ll - 2; q >= 0; q--) tail_up(E0(q), E1(q), R0(q), R1(q), E0(q + 1), E1(q + 1), nl >> q, nu2);
  if (GTOP) {
    tail_up(A.e0, A.e1, A.r0, A.r1, E0(0), E1(0), n0, nu2);
  } else {
    // LDS top level: the correction goes back to global memory
    const int half = n0 * n0 * n0 / 2;
    const T* e0 = E0(0);
    const T* e1 = E1(0);
    for (int t = tid * W; t < half; t += nt * W) {
      *reinterpret_cast<V*>(A.e0 + t) = *reinterpret_cast<const V*>(e0 + t);
      *reinterpret_cast<V*>(A.e1 + t) = *reinterpret_cast<const V*>(e1 + t);
    }
  }
}

template <typename T>
__device__ void Tail<T>::run(const Args& A, Grid) {
  // the stop flag is tested after the first loads are in flight (as in the
  // speculative upper-level launches); every wave reads the same flag
  const int done = A.ctl ? A.ctl->done : 0;
  if (A.n0 > kTailLdsMax)
    tail_run<T, true>(A, done);
  else
    tail_run<T, false>(A, done);
}

size_t tail_lds_bytes(int n0, int levels, size_t elem) {
  if (n0 > kTailLdsMax) {   // the top level stays in global memory
    n0 >>= 1;
    levels -= 1;
  }
  size_t tot = 0;
  for (int q = 0; q < levels; q++) {
    const size_t nq = (size_t)(n0 >> q);
    tot += 2 * nq * nq * nq;   // e0, e1, r0, r1 of nq^3/2 each
  }
  tot += (size_t)n0 * n0 * n0 / 2;   // red residuals
  return tot * elem;
}

// ---------------------------------------------------------------------------
// Field update (Supporting Information, numerical integration):
// phi^{k+1} = phi_p - (4 pi / h) y*, with y* projected to zero mean; the
// multiplier is pushed into the history on warm steps.
// ---------------------------------------------------------------------------
// Workgroups of the field update: 2,048 (eight per compute unit) keep every
// channel busy while the stop decision is made at most that many times.
constexpr int kPhiBlocks = 2048;
struct PhiUpdate {
  struct Args {
    int n3;
    double h;
    double *phi0, *phi1;
    const double *ya, *yb;
    double *yh0, *yh1, *yh2;
    float* phi32;
    Ctl* ctl;
    // the pending stop decision of the last outer residual, made by every
    // workgroup (the first records it); null: already made
    const double* dpart;
    int dnb, dn3, max_cycles;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void PhiUpdate::run(const Args& A, Grid G) {
  const int n4 = A.n3 >> 2;
  const double h = A.h;
  double* __restrict__ phi0 = A.phi0;
  double* __restrict__ phi1 = A.phi1;
  const double* __restrict__ ya = A.ya;
  const double* __restrict__ yb = A.yb;
  double* __restrict__ yh0 = A.yh0;
  double* __restrict__ yh1 = A.yh1;
  double* __restrict__ yh2 = A.yh2;
  float* __restrict__ phi32 = A.phi32;
  Ctl* ctl = A.ctl;
  int done, final_buf;
  double mean_y;
  if (A.dpart) {
    __shared__ double sh[32];
    __shared__ DecideOut out;
    outer_decide(ctl, A.dpart, A.dnb, A.dn3, A.max_cycles, G.b == 0, false, sh, &out);
    done = out.done;
    final_buf = out.final_buf;
    mean_y = out.mean_y;
  } else {
    done = ctl->done;
    final_buf = ctl->final_buf;
    mean_y = ctl->mean_y;
  }
  if (!done) return;   // enqueued ahead of the convergence check
  const int cold = ctl->cold;
  double* pk = ctl->k_idx ? phi1 : phi0;
  double* pkm1 = ctl->k_idx ? phi0 : phi1;
  const double* ysrc = final_buf ? yb : ya;
  double* const yh[3] = {yh0, yh1, yh2};
  double* ynew = yh[ctl->yh2];   // the oldest slot becomes the newest multiplier
  const double c4 = 4.0 * kPi / h;
  // four consecutive points per thread (two 16-byte loads per array)
  for (int g = G.b * kBlock + threadIdx.x; g < n4; g += G.g * kBlock) {
    const int t = 4 * g;
    const double2 y01 = *(const double2*)(ysrc + t), y23 = *(const double2*)(ysrc + t + 2);
    const double y[4] = {y01.x - mean_y, y01.y - mean_y, y23.x - mean_y, y23.y - mean_y};
    double phi[4];
    if (cold) {
      for (int i = 0; i < 4; i++) phi[i] = 0.0 - c4 * y[i];
      *(double2*)(pk + t) = make_double2(phi[0], phi[1]);
      *(double2*)(pk + t + 2) = make_double2(phi[2], phi[3]);
    } else {
      const double2 a01 = *(const double2*)(pk + t), a23 = *(const double2*)(pk + t + 2);
      const double2 b01 = *(const double2*)(pkm1 + t), b23 = *(const double2*)(pkm1 + t + 2);
      const double a[4] = {a01.x, a01.y, a23.x, a23.y}, b[4] = {b01.x, b01.y, b23.x, b23.y};
      for (int i = 0; i < 4; i++) phi[i] = (2.0 * a[i] - b[i]) - c4 * y[i];
      *(double2*)(ynew + t) = make_double2(y[0], y[1]);
      *(double2*)(ynew + t + 2) = make_double2(y[2], y[3]);
    }
    // pkm1 becomes phi^k after the rotation (a cold solve sets both)
    *(double2*)(pkm1 + t) = make_double2(phi[0], phi[1]);
    *(double2*)(pkm1 + t + 2) = make_double2(phi[2], phi[3]);
    if (phi32) *(float4*)(phi32 + t) = make_float4((float)phi[0], (float)phi[1], (float)phi[2], (float)phi[3]);
  }
}

// End of a step: rotate the potential and multiplier history (cold solves
// store no multiplier) and ramp the predictor order with the stored history.
struct Advance {
  struct Args {
    Ctl* ctl;
  };
  static constexpr int kThreads = 64;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void Advance::run(const Args& A, Grid) {
  Ctl* ctl = A.ctl;
  if (threadIdx.x != 0) return;
  if (ctl->cold) {
    ctl->n_yh = 0;
  } else {
    ctl->k_idx = 1 - ctl->k_idx;
    const int newest = ctl->yh2;
    ctl->yh2 = ctl->yh1;
    ctl->yh1 = ctl->yh0;
    ctl->yh0 = newest;
    ctl->n_yh = ctl->n_yh < 3 ? ctl->n_yh + 1 : 3;
  }
  ctl->cold = 0;
  ctl->m_eff = ctl->predictor < ctl->n_yh ? ctl->predictor : ctl->n_yh;
  ctl->steps += 1;
}

template <typename T>
__global__ void k_widen(int64_t count, const T* __restrict__ in, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = (double)in[t];
}

template <typename T>
__device__ __forceinline__ T cs_load(const T* __restrict__ c0, const T* __restrict__ c1, int n, int i, int j, int k) {
  const T* a = ((i + j + k) & 1) ? c1 : c0;
  return a[cs_idx(n, i, j, k)];
}

template <typename T>
__global__ void k_cs_to_nat(int n, const T* __restrict__ c0, const T* __restrict__ c1, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n * n) return;
  const int i = t % n, j = (t / n) % n, k = t / (n * n);
  out[t] = (double)cs_load(c0, c1, n, i, j, k);
}

template <typename T>
__global__ void k_nat_to_cs(int n, const double* __restrict__ in, T* __restrict__ c0, T* __restrict__ c1) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n * n) return;
  const int i = t % n, j = (t / n) % n, k = t / (n * n);
  T* d = ((i + j + k) & 1) ? c1 : c0;
  d[cs_idx(n, i, j, k)] = (T)in[t];
}

__global__ void k_sub_scalar(int64_t count, const double* __restrict__ in, double* __restrict__ out,
                             const double* __restrict__ sub) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = in[t] - *sub;
}

__global__ void k_set_open(Ctl* ctl) {
  ctl->done = 0;
  ctl->cycles = 0;
  ctl->status = 0;
  ctl->pending = 0;
}

// Vectorized sweeps: one thread per Vec<T>::W points, so half / W threads.
template <typename T>
int sweep_blocks(int n) {
  return blocks_for((int64_t)n * n * n / 2 / Vec<T>::W, kBlock);
}
// Levels up to this edge start speculatively (see keep_issued): a launch
// there moves a few MB at most, so a launch after convergence costs little
// more than its early return would.  Batched launches never speculate.
constexpr int kSpeculateMax = 128;
inline int speculate(int n) { return (n <= kSpeculateMax && g_recorder == nullptr) ? 1 : 0; }
template <typename T, int FIN>
hipError_t launch_sweep0(int n, T* r0, T* r1, T* e0, T* e1, Ctl* ctl, hipStream_t s) {
  if (speculate(n)) return go<SweepZero<T, FIN, 1>>({n, r0, r1, e0, e1, ctl}, sweep_blocks<T>(n), 0, s);
  return go<SweepZero<T, FIN, 0>>({n, r0, r1, e0, e1, ctl}, sweep_blocks<T>(n), 0, s);
}
template <typename T, int FIN>
hipError_t launch_half(int n, int colour, T* ec, const T* eo, const T* rc, Ctl* ctl, hipStream_t s) {
  if (speculate(n)) return go<Halfsweep<T, FIN, 1>>({n, colour, ec, eo, rc, ctl}, sweep_blocks<T>(n), 0, s);
  return go<Halfsweep<T, FIN, 0>>({n, colour, ec, eo, rc, ctl}, sweep_blocks<T>(n), 0, s);
}
template <typename T, int FIN>
hipError_t launch_restrict(int n, int red_only, const T* e0, const T* e1, const T* r0, const T* r1, T* rc0, T* rc1,
                           Ctl* ctl, hipStream_t s) {
  const int nc = n / 2;
  const int nb = blocks_for(nc * nc * nc, ResidRestrict<T, FIN, 0>::kThreads);
  if (red_only && restrict_col_on(n)) {
    const RestrictColGeo<T> cg(n, kRestrictColThreads);
    const int nj = nc / cg.JB;
    int nz = 1;
    while (nz < nc && nj * nz < 512) nz *= 2;
    return go<RestrictCol<T, FIN>>({n, red_only, e0, e1, r0, r1, rc0, rc1, ctl}, nj * nz,
                                   (size_t)cg.lds_elems() * sizeof(T), s);
  }
  if (red_only) {
    const int nbv = blocks_for(nc * nc * nc / Vec<T>::W, RestrictRed<T, FIN, 0>::kThreads);
    if (speculate(n)) return go<RestrictRed<T, FIN, 1>>({n, red_only, e0, e1, r0, r1, rc0, rc1, ctl}, nbv, 0, s);
    return go<RestrictRed<T, FIN, 0>>({n, red_only, e0, e1, r0, r1, rc0, rc1, ctl}, nbv, 0, s);
  }
  if (speculate(n)) return go<ResidRestrict<T, FIN, 1>>({n, red_only, e0, e1, r0, r1, rc0, rc1, ctl}, nb, 0, s);
  return go<ResidRestrict<T, FIN, 0>>({n, red_only, e0, e1, r0, r1, rc0, rc1, ctl}, nb, 0, s);
}
}  // namespace

bool post_sweeps_fused(const LevelBufs& b, bool fp64, int nu2) {
  return !fp64 && nu2 == 2 && (b.n == 512 || b.n == 256) && b.s0 && b.s1 && !g_recorder;
}

namespace {

hipError_t launch_post_sweeps(int n, const float* e1, const float* r0, const float* r1, float* s0, float* s1, Ctl* ctl,
                              hipStream_t s) {
  const int nj = n / PostGeo(n).JB;
  int nz = 1;
  while (nz < n && nj * nz < 256) nz *= 2;
  return go<PostSweeps>({n, e1, r0, r1, s0, s1, ctl}, nj * nz, (size_t)PostGeo(n).lds_floats() * 4, s);
}

// SweepRestrict applies to single systems' FP32 fine levels of 256^3 and
// 512^3 when the down leg is one sweep and the up leg starts with the
// black-only prolongation.
template <typename T>
bool sweep_restrict_on(int n, int nu1, int nu2) {
  return sizeof(T) == 4 && nu1 == 1 && nu2 >= 1 && n >= 256 && n <= 512 && !g_recorder;
}
hipError_t launch_sweep_restrict(int n, const float* r0, const float* r1, float* e1, float* rc0, float* rc1, Ctl* ctl,
                                 hipStream_t s) {
  const SweepRestrictGeo sg(n, kSweepRestrictThreads);
  const int nj = sg.nc / sg.JB;
  int nz = 1;
  while (nz < sg.nc && nj * nz < 512) nz *= 2;
  return go<SweepRestrict>({n, r0, r1, e1, rc0, rc1, ctl}, nj * nz, (size_t)sg.lds_floats() * 4, s);
}
template <typename T, int FIN>
hipError_t launch_prolong_black(int n, T* e1, const T* c0, const T* c1, Ctl* ctl, hipStream_t s) {
  if (n >= 256 && !g_recorder)
    return go<ProlongCol<T, FIN>>({n, e1, c0, c1, ctl}, blocks_for((int64_t)n * n / 2 / Vec<T>::W * (n / kProlongPlanes),
                                                                    kBlock), 0, s);
  if (speculate(n)) return go<ProlongBlack<T, FIN, 1>>({n, e1, c0, c1, ctl}, sweep_blocks<T>(n), 0, s);
  return go<ProlongBlack<T, FIN, 0>>({n, e1, c0, c1, ctl}, sweep_blocks<T>(n), 0, s);
}
template <typename T>
hipError_t launch_tail(const LevelBufs* lv, int levels, int tail, int nu1, int nu2, const double* green, Ctl* ctl,
                       hipStream_t s, const Decide* d = nullptr) {
  const int lt = levels - tail;
  return go<Tail<T>>({lv[tail].n, lt, nu1, nu2, (const T*)lv[tail].r0, (const T*)lv[tail].r1, (T*)lv[tail].e0,
                      (T*)lv[tail].e1, green, ctl, d ? d->partial : nullptr, d ? d->nb : 0, d ? d->n3 : 0,
                      d ? d->max_cycles : 0},
                     1, tail_lds_bytes(lv[tail].n, lt, sizeof(T)), s);
}

// Fused legs: LDS of one workgroup within the compute unit's 160 KiB.
constexpr size_t kFusedLdsCap = 160 * 1024;
constexpr int kFusedStepsMax = 8;

template <typename T>
bool fused_fits(int n, int ty, int tz, int S, int hb) {
  return ty > 0 && tz > 0 && n % ty == 0 && n % tz == 0 && (ty & 1) == 0 && (tz & 1) == 0 &&
         (n / 2) % Vec<T>::W == 0 && S >= 1 && S <= kFusedStepsMax &&
         FusedBox(n, ty, tz, S, hb).elems * sizeof(T) <= kFusedLdsCap;
}

// Both legs of level L fused (the down leg writes the buffers the up leg
// reads, so the two go together).
template <typename T>
bool fused_level(const LevelBufs& L, int nu1, int nu2) {
  return L.fty > 0 && L.d0 && L.d1 && nu1 >= 1 && nu2 >= 1 && fused_fits<T>(L.n, L.fty, L.ftz, 2 * nu1 - 1, 0) &&
         fused_fits<T>(L.n, L.fty, L.ftz, 2 * nu2, 0);
}
// The fused down leg of L also restricts (its wider box fits in LDS).
template <typename T>
bool fused_restricts(const LevelBufs& L, int nu1, int nu2) {
  return fused_level<T>(L, nu1, nu2) && fused_fits<T>(L.n, L.fty, L.ftz, 2 * nu1 - 1, 2);
}

template <typename T, int UP, int FIN, int RST>
hipError_t launch_fused_t(int n, int ty, int tz, int S, const T* r0, const T* r1, const T* src1, const T* ec0,
                          const T* ec1, T* out0, T* out1, T* rc0, T* rc1, Ctl* ctl, hipStream_t s) {
  const int hb = RST ? 2 : 0;
  if (!fused_fits<T>(n, ty, tz, S, hb)) return hipErrorInvalidValue;
  const int grid = (n / ty) * (n / tz);
  const size_t lds = FusedBox(n, ty, tz, S, hb).elems * sizeof(T);
  return go<Fused<T, UP, FIN, RST>>({n, ty, tz, S, r0, r1, src1, ec0, ec1, out0, out1, rc0, rc1, ctl}, grid, lds, s);
}

// Down leg of level L: first sweep from zero and nu1 - 1 pairs into d0/d1;
// with RST also the restricted residual into the coarse level C's rhs.
template <typename T, int FIN, int RST>
hipError_t launch_fused_down(const LevelBufs& L, const LevelBufs& C, int nu1, Ctl* ctl, hipStream_t s) {
  return launch_fused_t<T, 0, FIN, RST>(L.n, L.fty, L.ftz, 2 * nu1 - 1, (const T*)L.r0, (const T*)L.r1, nullptr,
                                        nullptr, nullptr, (T*)L.d0, (T*)L.d1, RST ? (T*)C.r0 : nullptr,
                                        RST ? (T*)C.r1 : nullptr, ctl, s);
}
// Up leg of level L: black-point correction from the coarse level C, then
// nu2 pairs, from d1 into e0/e1.
template <typename T, int FIN>
hipError_t launch_fused_up(const LevelBufs& L, const LevelBufs& C, int nu2, Ctl* ctl, hipStream_t s) {
  return launch_fused_t<T, 1, FIN, 0>(L.n, L.fty, L.ftz, 2 * nu2, (const T*)L.r0, (const T*)L.r1, (const T*)L.d1,
                                      (const T*)C.e0, (const T*)C.e1, (T*)L.e0, (T*)L.e1, nullptr, nullptr, ctl, s);
}

#define P3MZ_LAUNCH(...)             \
  do {                               \
    hipError_t e_ = (__VA_ARGS__);   \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// Sequence keys of the V-cycle launches (merge keys of batched systems):
// level l from the finest going down, the tail, then the levels going up in
// reverse, so systems with fewer levels keep their own order in a batch.
// Sub-keys: 0..33 sweeps and prolongation (up: 0 black-point prolongation,
// then 2 + 2 it + colour), 60 fused leg, 62 zero fill, 63 restriction /
// plain prolongation.
inline uint32_t key_down(int l, int sub) { return 1000u + 64u * (uint32_t)l + (uint32_t)sub; }
inline uint32_t key_up(int l, int sub) { return 3000u + 64u * (uint32_t)(P3MZ_MAX_LEVELS - 1 - l) + (uint32_t)sub; }
constexpr uint32_t kKeyTail = 2100u;

template <typename T>
hipError_t vcycle_impl(const LevelBufs* lv, int levels, int tail, int nu1, int nu2, const double* green,
                       Ctl* ctl, hipStream_t s, const Decide* decide) {
  const double ts = sizeof(T);
  for (int l = 0; l < tail; l++) {
    const int n = lv[l].n, half = n * n * n / 2;
    const double n3 = (double)n * n * n;
    T *e0 = (T*)lv[l].e0, *e1 = (T*)lv[l].e1, *r0 = (T*)lv[l].r0, *r1 = (T*)lv[l].r1;
    if (sweep_restrict_on<T>(n, nu1, nu2)) {
      // the single pre-smoothing sweep and the restriction in one walk
      rec_key(key_down(l, 63));
      kt_begin(KT_RESTRICT, l, s);
      P3MZ_LAUNCH(launch_sweep_restrict(n, (const float*)r0, (const float*)r1, (float*)e1, (float*)lv[l + 1].r0,
                                        (float*)lv[l + 1].r1, ctl, s));
      kt_end(KT_RESTRICT, l, 1.625 * ts * n3, s);
      continue;
    }
    if (fused_restricts<T>(lv[l], nu1, nu2)) {
      rec_key(key_down(l, 61));
      kt_begin(KT_FUSED_DOWN, l, s);
      P3MZ_LAUNCH(l == 0 ? launch_fused_down<T, 1, 1>(lv[l], lv[l + 1], nu1, ctl, s)
                         : launch_fused_down<T, 0, 1>(lv[l], lv[l + 1], nu1, ctl, s));
      kt_end(KT_FUSED_DOWN, l, 2.125 * ts * n3, s);
      continue;   // restricted in the same launch
    }
    if (fused_level<T>(lv[l], nu1, nu2)) {
      rec_key(key_down(l, 60));
      kt_begin(KT_FUSED_DOWN, l, s);
      P3MZ_LAUNCH(l == 0 ? launch_fused_down<T, 1, 0>(lv[l], lv[l + 1], nu1, ctl, s)
                         : launch_fused_down<T, 0, 0>(lv[l], lv[l + 1], nu1, ctl, s));
      kt_end(KT_FUSED_DOWN, l, 2.0 * ts * n3, s);
      // the restriction reads the down leg's result
      e0 = (T*)lv[l].d0;
      e1 = (T*)lv[l].d1;
    } else if (nu1 >= 1) {
      rec_key(key_down(l, 0));
      kt_begin(KT_SWEEP0, l, s);
      P3MZ_LAUNCH(l == 0 ? launch_sweep0<T, 1>(n, r0, r1, e0, e1, ctl, s) : launch_sweep0<T, 0>(n, r0, r1, e0, e1, ctl, s));
      kt_end(KT_SWEEP0, l, 2.0 * ts * n3, s);
      for (int it = 1; it < nu1; it++) {
        for (int colour = 0; colour < 2; colour++) {
          T* ec = colour ? e1 : e0;
          const T* eo = colour ? e0 : e1;
          const T* rc = colour ? r1 : r0;
          rec_key(key_down(l, 1 + 2 * (it - 1) + colour));
          kt_begin(KT_HALFSWEEP, l, s);
          P3MZ_LAUNCH(l == 0 ? launch_half<T, 1>(n, colour, ec, eo, rc, ctl, s)
                             : launch_half<T, 0>(n, colour, ec, eo, rc, ctl, s));
          kt_end(KT_HALFSWEEP, l, 1.5 * ts * n3, s);
        }
      }
    } else {
      rec_key(key_down(l, 62));
      P3MZ_LAUNCH(go<FillZero<T>>({(int64_t)half, e0, e1, ctl}, blocks_for(half, kBlock), 0, s));
    }
    rec_key(key_down(l, 63));
    kt_begin(KT_RESTRICT, l, s);
    T *c0 = (T*)lv[l + 1].r0, *c1 = (T*)lv[l + 1].r1;
    P3MZ_LAUNCH(l == 0 ? launch_restrict<T, 1>(n, nu1 >= 1, e0, e1, r0, r1, c0, c1, ctl, s)
                       : launch_restrict<T, 0>(n, nu1 >= 1, e0, e1, r0, r1, c0, c1, ctl, s));
    // red-only restriction: e0, e1, r0 read, the coarse right-hand side written
    kt_end(KT_RESTRICT, l, (nu1 >= 1 ? 1.625 : 2.125) * ts * n3, s);
  }
  {
    const double nt3 = (double)lv[tail].n * lv[tail].n * lv[tail].n;
    rec_key(kKeyTail);
    kt_begin(KT_TAIL, 0, s);
    P3MZ_LAUNCH(launch_tail<T>(lv, levels, tail, nu1, nu2, green, ctl, s, decide));
    kt_end(KT_TAIL, 0, 2.0 * ts * nt3, s);
  }
  for (int l = tail - 1; l >= 0; l--) {
    const int n = lv[l].n, half = n * n * n / 2, nb = blocks_for(half, kBlock);
    const double n3 = (double)n * n * n;
    T *e0 = (T*)lv[l].e0, *e1 = (T*)lv[l].e1, *r0 = (T*)lv[l].r0, *r1 = (T*)lv[l].r1;
    // the coarse level's correction (in s0/s1 when its post-smoothing ran as one walk)
    const T* c0 = (const T*)cycle_e0(lv[l + 1], sizeof(T) == 8, nu2);
    const T* c1 = (const T*)cycle_e1(lv[l + 1], sizeof(T) == 8, nu2);
    if (fused_level<T>(lv[l], nu1, nu2)) {
      rec_key(key_up(l, 60));
      kt_begin(KT_FUSED_UP, l, s);
      P3MZ_LAUNCH(l == 0 ? launch_fused_up<T, 1>(lv[l], lv[l + 1], nu2, ctl, s)
                         : launch_fused_up<T, 0>(lv[l], lv[l + 1], nu2, ctl, s));
      kt_end(KT_FUSED_UP, l, 2.625 * ts * n3, s);
    } else if (nu2 >= 1) {
      rec_key(key_up(l, 0));
      kt_begin(KT_PROLONG, l, s);
      P3MZ_LAUNCH(l == 0 ? launch_prolong_black<T, 1>(n, e1, c0, c1, ctl, s)
                         : launch_prolong_black<T, 0>(n, e1, c0, c1, ctl, s));
      kt_end(KT_PROLONG, l, 1.125 * ts * n3, s);
      if (post_sweeps_fused(lv[l], sizeof(T) == 8, nu2)) {
        // both sweeps in one walk; the level's correction goes to s0/s1
        rec_key(key_up(l, 2));
        kt_begin(KT_HALFSWEEP, l, s);
        P3MZ_LAUNCH(launch_post_sweeps(n, (const float*)e1, (const float*)r0, (const float*)r1, (float*)lv[l].s0,
                                       (float*)lv[l].s1, ctl, s));
        kt_end(KT_HALFSWEEP, l, 2.5 * ts * n3, s);
        continue;
      }
      for (int it = 0; it < nu2; it++) {
        for (int colour = 0; colour < 2; colour++) {
          T* ec = colour ? e1 : e0;
          const T* eo = colour ? e0 : e1;
          const T* rc = colour ? r1 : r0;
          rec_key(key_up(l, 2 + 2 * it + colour));
          kt_begin(KT_HALFSWEEP, l, s);
          P3MZ_LAUNCH(l == 0 ? launch_half<T, 1>(n, colour, ec, eo, rc, ctl, s)
                             : launch_half<T, 0>(n, colour, ec, eo, rc, ctl, s));
          kt_end(KT_HALFSWEEP, l, 1.5 * ts * n3, s);
        }
      }
    } else {
      rec_key(key_up(l, 63));
      kt_begin(KT_PROLONG, l, s);
      P3MZ_LAUNCH(go<ProlongAdd<T>>({n, e0, e1, c0, c1, ctl}, nb, 0, s));
      kt_end(KT_PROLONG, l, 2.125 * ts * n3, s);
    }
  }
  return hipSuccess;
}

// One launch of a finest-level V-cycle kernel family on the current buffers
// (for back-to-back timing); returns its algorithmic bytes.
template <typename T>
hipError_t one_kernel(int kid, const LevelBufs* lv, int levels, int tail, int nu1, int nu2, const double* green,
                      Ctl* ctl, hipStream_t s, double* bytes) {
  const int n = lv[0].n, half = n * n * n / 2, nb = blocks_for(half, kBlock);
  const double n3 = (double)n * n * n, ts = sizeof(T);
  T *e0 = (T*)lv[0].e0, *e1 = (T*)lv[0].e1, *r0 = (T*)lv[0].r0, *r1 = (T*)lv[0].r1;
  if ((kid == KT_HALFSWEEP || kid == KT_SWEEP0) && (n / 2) % Vec<T>::W != 0) return hipErrorInvalidValue;
  switch (kid) {
    case KT_HALFSWEEP:
      *bytes = 1.5 * ts * n3;
      return launch_half<T, 1>(n, 0, e0, e1, r0, ctl, s);
    case KT_SWEEP0:
      *bytes = 2.0 * ts * n3;
      return launch_sweep0<T, 1>(n, r0, r1, e0, e1, ctl, s);
    case KT_RESTRICT:
      if (tail == 0) return hipErrorInvalidValue;
      *bytes = (nu1 >= 1 ? 1.625 : 2.125) * ts * n3;
      return launch_restrict<T, 1>(n, nu1 >= 1, e0, e1, r0, r1, (T*)lv[1].r0, (T*)lv[1].r1, ctl, s);
    case KT_PROLONG:
      if (tail == 0) return hipErrorInvalidValue;
      *bytes = 1.125 * ts * n3;
      return launch_prolong_black<T, 1>(n, e1, (const T*)lv[1].e0, (const T*)lv[1].e1, ctl, s);
    case KT_FUSED_DOWN:
      if (tail == 0 || !fused_level<T>(lv[0], nu1, nu2)) return hipErrorInvalidValue;
      if (fused_restricts<T>(lv[0], nu1, nu2)) {
        *bytes = 2.125 * ts * n3;
        return launch_fused_down<T, 1, 1>(lv[0], lv[1], nu1, ctl, s);
      }
      *bytes = 2.0 * ts * n3;
      return launch_fused_down<T, 1, 0>(lv[0], lv[1], nu1, ctl, s);
    case KT_FUSED_UP:
      if (tail == 0 || !fused_level<T>(lv[0], nu1, nu2)) return hipErrorInvalidValue;
      *bytes = 2.625 * ts * n3;
      return launch_fused_up<T, 1>(lv[0], lv[1], nu2, ctl, s);
    case KT_TAIL:
      *bytes = 2.0 * ts * (double)lv[tail].n * lv[tail].n * lv[tail].n;
      return launch_tail<T>(lv, levels, tail, nu1, nu2, green, ctl, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

// Smoothing launch shapes (W lines per workgroup, R outputs per thread);
// variant 0 is the default, the others are candidates for the autotuner.
constexpr int kSmoothTiles[][2] = {{16, 8}, {32, 8}, {8, 8}, {32, 4}, {16, 4}, {8, 4}, {4, 8}};
constexpr int kSmoothTileCount = (int)(sizeof(kSmoothTiles) / sizeof(kSmoothTiles[0]));
// dynamic LDS of one smoothing workgroup: four fit on a compute unit, so
// enough waves are in flight to cover the memory latency
constexpr size_t kSmoothLdsCap = 40 * 1024;

namespace {
// Segment length of one axis' pass: the longest power-of-two piece of a
// line (whole lines first) whose workgroup fits in kSmoothLdsCap; 0 if none.
int smooth_segment(int n, int W, int R, int ntaps, int axis) {
  for (int S = n; S >= R; S >>= 1)
    if ((size_t)SmoothLds(axis, W, R, ntaps, S).total * sizeof(double) <= kSmoothLdsCap) return S;
  return 0;
}

// (The segment is sized for FP64 elements; an FP32 pass uses the same
// segment in half the LDS.)
template <typename T, int W, int R>
hipError_t smooth_wr(int n, int axis, int ntaps, int half, const T* tp, const T* ip, T* op, hipStream_t s) {
  const int S = smooth_segment(n, W, R, ntaps, axis);
  if (S == 0) return hipErrorInvalidValue;
  const int nseg = n / S;
  const int grid = (axis == 0 ? (int)((size_t)n * n / W) : (n / W) * n) * nseg;
  const size_t lds = (size_t)SmoothLds(axis, W, R, ntaps, S, 16 / (int)sizeof(T)).total * sizeof(T);
  if (axis == 0) return go<Smooth<T, 0, W, R>>({n, ntaps, half, S, tp, ip, op}, grid, lds, s);
  if (axis == 1) return go<Smooth<T, 1, W, R>>({n, ntaps, half, S, tp, ip, op}, grid, lds, s);
  return go<Smooth<T, 2, W, R>>({n, ntaps, half, S, tp, ip, op}, grid, lds, s);
}

template <typename T, int W, int R>
hipError_t smooth_allow_t() {
  P3MZ_LAUNCH(allow_lds<Smooth<T, 0, W, R>>((int)kSmoothLdsCap));
  P3MZ_LAUNCH(allow_lds<Smooth<T, 1, W, R>>((int)kSmoothLdsCap));
  return allow_lds<Smooth<T, 2, W, R>>((int)kSmoothLdsCap);
}
template <int W, int R>
hipError_t smooth_allow() {
  P3MZ_LAUNCH((smooth_allow_t<double, W, R>()));
  return smooth_allow_t<float, W, R>();
}

template <typename T>
hipError_t smooth_t(int n, int axis, int tile, int ntaps, int half, const T* tp, const T* ip, T* op, hipStream_t s) {
  switch (tile) {
    case 0: return smooth_wr<T, 16, 8>(n, axis, ntaps, half, tp, ip, op, s);
    case 1: return smooth_wr<T, 32, 8>(n, axis, ntaps, half, tp, ip, op, s);
    case 2: return smooth_wr<T, 8, 8>(n, axis, ntaps, half, tp, ip, op, s);
    case 3: return smooth_wr<T, 32, 4>(n, axis, ntaps, half, tp, ip, op, s);
    case 4: return smooth_wr<T, 16, 4>(n, axis, ntaps, half, tp, ip, op, s);
    case 5: return smooth_wr<T, 8, 4>(n, axis, ntaps, half, tp, ip, op, s);
    default: return smooth_wr<T, 4, 8>(n, axis, ntaps, half, tp, ip, op, s);
  }
}
}  // namespace

int smooth_tile_count() { return kSmoothTileCount; }

bool smooth_tile_ok(int tile, int n, int ntaps) {
  if (tile < 0 || tile >= kSmoothTileCount) return false;
  const int W = kSmoothTiles[tile][0], R = kSmoothTiles[tile][1];
  return n % W == 0 && n % R == 0 && smooth_segment(n, W, R, ntaps, 0) > 0 && smooth_segment(n, W, R, ntaps, 1) > 0;
}

void smooth_tile_shape(int tile, int* w, int* r) {
  *w = kSmoothTiles[tile][0];
  *r = kSmoothTiles[tile][1];
}

hipError_t launch_smooth(bool fp64, int n, int axis, int tile, int ntaps, int half, const void* taps, const void* in,
                         void* out, hipStream_t s) {
  if (!smooth_tile_ok(tile, n, ntaps)) return hipErrorInvalidValue;
  if (fp64)
    return smooth_t<double>(n, axis, tile, ntaps, half, (const double*)taps, (const double*)in, (double*)out, s);
  return smooth_t<float>(n, axis, tile, ntaps, half, (const float*)taps, (const float*)in, (float*)out, s);
}

// Every smoothing kernel may use up to kSmoothLdsCap of dynamic LDS.
hipError_t smooth_configure() {
  static bool granted = false;
  if (granted) return hipSuccess;
  P3MZ_LAUNCH(smooth_allow<16, 8>());
  P3MZ_LAUNCH(smooth_allow<32, 8>());
  P3MZ_LAUNCH(smooth_allow<8, 8>());
  P3MZ_LAUNCH(smooth_allow<32, 4>());
  P3MZ_LAUNCH(smooth_allow<16, 4>());
  P3MZ_LAUNCH(smooth_allow<8, 4>());
  P3MZ_LAUNCH(smooth_allow<4, 8>());
  granted = true;
  return hipSuccess;
}

hipError_t launch_sigma(int n, double h, bool qs32, const void* qs, const double* phi0, const double* phi1,
                        const double* yb0, const double* yb1, const double* yb2, double* sigma, double* y,
                        double tol, int tol_mode, double* partial, Ctl* ctl, hipStream_t s, bool finalize,
                        int stencil) {
  const int n3 = n * n * n, nb = red_blocks(n3 / 4);   // four points per thread
  const float* q32 = (const float*)qs;
  const double* q64 = (const double*)qs;
  if (stencil == 1) {
    if (qs32)
      P3MZ_LAUNCH(go<SigmaHO<float>>({n, h, q32, phi0, phi1, yb0, yb1, yb2, sigma, y, partial, ctl, nb}, nb, 0, s));
    else
      P3MZ_LAUNCH(go<SigmaHO<double>>({n, h, q64, phi0, phi1, yb0, yb1, yb2, sigma, y, partial, ctl, nb}, nb, 0, s));
  } else if (col_walk_on(n)) {
    const int grid = col_grid(kColThreads, n, kColPerCu);
    const size_t lds = col_lds_bytes(kColThreads, n);
    if (qs32)
      P3MZ_LAUNCH(go<Sigma<float, kColThreads>>({n, h, q32, phi0, phi1, yb0, yb1, yb2, sigma, y, partial, ctl, nb},
                                                grid, lds, s));
    else
      P3MZ_LAUNCH(go<Sigma<double, kColThreads>>({n, h, q64, phi0, phi1, yb0, yb1, yb2, sigma, y, partial, ctl, nb},
                                                 grid, lds, s));
  } else if (qs32) {
    P3MZ_LAUNCH(go<Sigma<float>>({n, h, q32, phi0, phi1, yb0, yb1, yb2, sigma, y, partial, ctl, nb}, nb, 0, s));
  } else {
    P3MZ_LAUNCH(go<Sigma<double>>({n, h, q64, phi0, phi1, yb0, yb1, yb2, sigma, y, partial, ctl, nb}, nb, 0, s));
  }
  if (!finalize) return hipSuccess;
  return go<FinSigma>({nb, n3, tol_mode, tol, partial, ctl}, 1, 0, s);
}

hipError_t launch_outer(bool fp64, int n, int first, int max_cycles, const double* sigma, double* y0, double* y1,
                        const void* e0, const void* e1, void* r0, void* r1, double* partial, Ctl* ctl,
                        hipStream_t s, bool finalize, const double* spart, double tol, int tol_mode, int stencil) {
  const int n3 = n * n * n, nb = red_blocks(n3 / 4);   // four points per thread (sigma's partial count too)
  if (!first) spart = nullptr;
  const double *d0 = (const double*)e0, *d1 = (const double*)e1;
  const float *f0 = (const float*)e0, *f1 = (const float*)e1;
  double *dr0 = (double*)r0, *dr1 = (double*)r1;
  float *fr0 = (float*)r0, *fr1 = (float*)r1;
  if (stencil == 1 && fp64)
    P3MZ_LAUNCH(go<OuterHO<double>>(
        {n, first, sigma, y0, y1, d0, d1, dr0, dr1, partial, ctl, spart, tol_mode, tol, nb}, nb, 0, s));
  else if (stencil == 1)
    P3MZ_LAUNCH(go<OuterHO<float>>(
        {n, first, sigma, y0, y1, f0, f1, fr0, fr1, partial, ctl, spart, tol_mode, tol, nb}, nb, 0, s));
  else if (col_walk_on(n)) {
    const int grid = col_grid(kColThreads, n, kColPerCu);
    const size_t lds = col_lds_bytes(kColThreads, n);
    if (fp64)
      P3MZ_LAUNCH(go<Outer<double, kColThreads>>(
          {n, first, sigma, y0, y1, d0, d1, dr0, dr1, partial, ctl, spart, tol_mode, tol, nb}, grid, lds, s));
    else
      P3MZ_LAUNCH(go<Outer<float, kColThreads>>(
          {n, first, sigma, y0, y1, f0, f1, fr0, fr1, partial, ctl, spart, tol_mode, tol, nb}, grid, lds, s));
  } else if (fp64)
    P3MZ_LAUNCH(go<Outer<double>>(
        {n, first, sigma, y0, y1, d0, d1, dr0, dr1, partial, ctl, spart, tol_mode, tol, nb}, nb, 0, s));
  else
    P3MZ_LAUNCH(go<Outer<float>>(
        {n, first, sigma, y0, y1, f0, f1, fr0, fr1, partial, ctl, spart, tol_mode, tol, nb}, nb, 0, s));
  if (!finalize) return hipSuccess;
  return go<FinOuter>({max_cycles, nb, n3, partial, ctl}, 1, 0, s);
}

// ---------------------------------------------------------------------------
// Persistent form of a batch's finest-level sweeps, built to measure it
// against one batched launch per sweep: one launch runs `phases`
// half-sweeps (colours alternating) on every system.  The tasks (phase,
// system, tile) are numbered phase-major and workgroup b of a grid that fits
// on the device at once takes tasks b, b + G, b + 2G, ... in order; a task of
// phase p waits until every tile of its own system's phase p-1 is done (a
// per-system device barrier with acquire/release fences at agent scope), so
// systems advance independently instead of meeting at kernel boundaries.
// Every wait is on tasks with smaller numbers, held by resident workgroups
// that take their tasks in increasing order, so the waits end; a bounded
// spin sets an error flag instead of waiting forever.  The task loop's
// bounds are kernel arguments and the block index (uniform): no workgroup
// barrier sits in a loop whose exit depends on a value read from memory.
// ---------------------------------------------------------------------------
template <typename T>
struct PersistSys {
  typename Halfsweep<T, 1, 0>::Args a[2];   // red, black
  int grid, off;                             // tiles per phase, first task of the system in a phase
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_persist_halfsweeps(const PersistSys<T>* __restrict__ sys, int n_sys,
                                                                int per_phase, int phases, int* __restrict__ work) {
  // work[1]: error flag, work[2 + r * phases + p]: finished tiles of system r, phase p
  const int total = per_phase * phases;
  for (int task = blockIdx.x; task < total; task += gridDim.x) {
    const int p = task / per_phase, w = task - p * per_phase;
    int lo = 0, hi = n_sys - 1;   // the system whose tasks hold w
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sys[mid].off <= w) lo = mid;
      else hi = mid - 1;
    }
    const PersistSys<T>& S = sys[lo];
    if (p > 0 && threadIdx.x == 0) {
      int* dep = &work[2 + lo * phases + p - 1];
      int spins = 0;
      while (__hip_atomic_load(dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < S.grid && spins < (1 << 22)) {
        __builtin_amdgcn_s_sleep(2);
        spins++;
      }
      if (spins >= (1 << 22)) atomicExch(&work[1], 1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see the other XCDs' stores
    }
    __syncthreads();
    Halfsweep<T, 1, 0>::run(S.a[p & 1], Grid{w - S.off, S.grid});
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(&work[2 + lo * phases + p], 1);
    }
  }
}

__global__ void k_zero_ints(int* __restrict__ a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0;
}

hipError_t persist_halfsweeps(bool fp64, const LevelBufs* const* lv0, Ctl* const* ctls, int n_sys, int phases,
                              void* d_sys, int* d_work, int grid, hipStream_t s, size_t* sys_bytes, bool upload) {
  const size_t elem = fp64 ? sizeof(PersistSys<double>) : sizeof(PersistSys<float>);
  *sys_bytes = elem * (size_t)n_sys;
  int per_phase = 0;
  if (upload) {
    std::vector<unsigned char> host(*sys_bytes);
    for (int r = 0; r < n_sys; r++) {
      const LevelBufs& f = *lv0[r];
      if (fp64) {
        PersistSys<double> x{};
        for (int c = 0; c < 2; c++)
          x.a[c] = {f.n, c, (double*)(c ? f.e1 : f.e0), (const double*)(c ? f.e0 : f.e1),
                    (const double*)(c ? f.r1 : f.r0), ctls[r]};
        x.grid = sweep_blocks<double>(f.n);
        x.off = per_phase;
        per_phase += x.grid;
        memcpy(host.data() + elem * r, &x, elem);
      } else {
        PersistSys<float> x{};
        for (int c = 0; c < 2; c++)
          x.a[c] = {f.n, c, (float*)(c ? f.e1 : f.e0), (const float*)(c ? f.e0 : f.e1),
                    (const float*)(c ? f.r1 : f.r0), ctls[r]};
        x.grid = sweep_blocks<float>(f.n);
        x.off = per_phase;
        per_phase += x.grid;
        memcpy(host.data() + elem * r, &x, elem);
      }
    }
    P3MZ_LAUNCH(hipMemcpy(d_sys, host.data(), host.size(), hipMemcpyHostToDevice));
  } else {
    for (int r = 0; r < n_sys; r++) per_phase += fp64 ? sweep_blocks<double>(lv0[r]->n) : sweep_blocks<float>(lv0[r]->n);
  }
  const int nwork = 2 + n_sys * phases;
  hipLaunchKernelGGL(k_zero_ints, dim3((nwork + 255) / 256), dim3(256), 0, s, d_work, nwork);
  P3MZ_LAUNCH(hipGetLastError());
  if (fp64)
    hipLaunchKernelGGL(k_persist_halfsweeps<double>, dim3(grid), dim3(kBlock), 0, s, (const PersistSys<double>*)d_sys,
                       n_sys, per_phase, phases, d_work);
  else
    hipLaunchKernelGGL(k_persist_halfsweeps<float>, dim3(grid), dim3(kBlock), 0, s, (const PersistSys<float>*)d_sys,
                       n_sys, per_phase, phases, d_work);
  return hipGetLastError();
}

size_t persist_sys_bytes(bool fp64, int n_sys) {
  return (fp64 ? sizeof(PersistSys<double>) : sizeof(PersistSys<float>)) * (size_t)n_sys;
}

int persist_grid() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist_halfsweeps<float>, kBlock, 0) != hipSuccess)
    return 0;
  return cus * std::max(1, per_cu);
}

hipError_t launch_vcycle(bool fp64, const LevelBufs* lv, int levels, int tail, int nu1, int nu2,
                         const double* green, Ctl* ctl, hipStream_t s, const Decide* decide) {
  return fp64 ? vcycle_impl<double>(lv, levels, tail, nu1, nu2, green, ctl, s, decide)
              : vcycle_impl<float>(lv, levels, tail, nu1, nu2, green, ctl, s, decide);
}

hipError_t launch_vcycle_kernel(bool fp64, int kid, const LevelBufs* lv, int levels, int tail, int nu1, int nu2,
                                const double* green, Ctl* ctl, hipStream_t s, double* bytes) {
  return fp64 ? one_kernel<double>(kid, lv, levels, tail, nu1, nu2, green, ctl, s, bytes)
              : one_kernel<float>(kid, lv, levels, tail, nu1, nu2, green, ctl, s, bytes);
}

hipError_t tail_configure(bool fp64, int n_tail, int levels_tail, size_t* lds_bytes) {
  static int granted[2] = {0, 0};
  const size_t b = tail_lds_bytes(n_tail, levels_tail, fp64 ? 8 : 4);
  *lds_bytes = b;
  if ((int)b <= granted[fp64]) return hipSuccess;
  P3MZ_LAUNCH(fp64 ? allow_lds<Tail<double>>((int)b) : allow_lds<Tail<float>>((int)b));
  granted[fp64] = (int)b;
  return hipSuccess;
}

int fused_tile(int n) { return n >= 64 ? 4 : 2; }

namespace {
template <typename T, int UP, int RST>
hipError_t fused_allow() {
  P3MZ_LAUNCH(allow_lds<Fused<T, UP, 0, RST>>((int)kFusedLdsCap));
  return allow_lds<Fused<T, UP, 1, RST>>((int)kFusedLdsCap);
}
}  // namespace

hipError_t fused_configure() {
  static bool done = false;
  if (done) return hipSuccess;
  P3MZ_LAUNCH((fused_allow<float, 0, 0>()));
  P3MZ_LAUNCH((fused_allow<float, 0, 1>()));
  P3MZ_LAUNCH((fused_allow<float, 1, 0>()));
  P3MZ_LAUNCH((fused_allow<double, 0, 0>()));
  P3MZ_LAUNCH((fused_allow<double, 0, 1>()));
  P3MZ_LAUNCH((fused_allow<double, 1, 0>()));
  // the shared-row column walk of sigma_p and the outer residual
  const int col = (int)col_lds_bytes(kColThreads, 512);
  P3MZ_LAUNCH((allow_lds<Sigma<float, kColThreads>>(col)));
  P3MZ_LAUNCH((allow_lds<Sigma<double, kColThreads>>(col)));
  P3MZ_LAUNCH((allow_lds<Outer<float, kColThreads>>(col)));
  P3MZ_LAUNCH((allow_lds<Outer<double, kColThreads>>(col)));
  // the two post-smoothing sweeps as one walk
  P3MZ_LAUNCH((allow_lds<PostSweeps>(std::max(PostGeo(512).lds_floats(), PostGeo(256).lds_floats()) * 4)));
  // the column-walk restriction and the fused first sweep and restriction
  P3MZ_LAUNCH((allow_lds<SweepRestrict>(std::max(SweepRestrictGeo(256, kSweepRestrictThreads).lds_floats(),
                                                  SweepRestrictGeo(512, kSweepRestrictThreads).lds_floats()) * 4)));
  const int rf = RestrictColGeo<float>(512, kRestrictColThreads).lds_elems() * 4;
  const int rd = RestrictColGeo<double>(512, kRestrictColThreads).lds_elems() * 8;
  P3MZ_LAUNCH((allow_lds<RestrictCol<float, 0>>(rf)));
  P3MZ_LAUNCH((allow_lds<RestrictCol<float, 1>>(rf)));
  P3MZ_LAUNCH((allow_lds<RestrictCol<double, 0>>(rd)));
  P3MZ_LAUNCH((allow_lds<RestrictCol<double, 1>>(rd)));
  done = true;
  return hipSuccess;
}

hipError_t launch_phi_update(int n, double h, double* phi0, double* phi1, const double* ya, const double* yb,
                             double* yh0, double* yh1, double* yh2, float* phi32, Ctl* ctl, hipStream_t s,
                             const Decide* d) {
  const int n3 = n * n * n;
  // a capped grid: every workgroup makes the stop decision once (reading
  // the outer residual's partials), then streams four points per thread
  const int nb = std::max(1, std::min(blocks_for(n3 / 4, kBlock), kPhiBlocks));
  return go<PhiUpdate>({n3, h, phi0, phi1, ya, yb, yh0, yh1, yh2, phi32, ctl, d ? d->partial : nullptr,
                        d ? d->nb : 0, d ? d->n3 : 0, d ? d->max_cycles : 0},
                       nb, 0, s);
}

hipError_t launch_advance(Ctl* ctl, hipStream_t s) { return go<Advance>({ctl}, 1, 0, s); }

hipError_t launch_widen(bool fp64, int64_t count, const void* in, double* out, hipStream_t s) {
  const int nb = blocks_for(count, kBlock);
  if (fp64)
    hipLaunchKernelGGL(k_widen<double>, dim3(nb), dim3(kBlock), 0, s, count, (const double*)in, out);
  else
    hipLaunchKernelGGL(k_widen<float>, dim3(nb), dim3(kBlock), 0, s, count, (const float*)in, out);
  return hipGetLastError();
}

hipError_t launch_cs_to_nat(bool fp64, int n, const void* c0, const void* c1, double* out, hipStream_t s) {
  const int nb = blocks_for(n * n * n, kBlock);
  if (fp64)
    hipLaunchKernelGGL(k_cs_to_nat<double>, dim3(nb), dim3(kBlock), 0, s, n, (const double*)c0, (const double*)c1, out);
  else
    hipLaunchKernelGGL(k_cs_to_nat<float>, dim3(nb), dim3(kBlock), 0, s, n, (const float*)c0, (const float*)c1, out);
  return hipGetLastError();
}

hipError_t launch_nat_to_cs(bool fp64, int n, const double* in, void* c0, void* c1, hipStream_t s) {
  const int nb = blocks_for(n * n * n, kBlock);
  if (fp64)
    hipLaunchKernelGGL(k_nat_to_cs<double>, dim3(nb), dim3(kBlock), 0, s, n, in, (double*)c0, (double*)c1);
  else
    hipLaunchKernelGGL(k_nat_to_cs<float>, dim3(nb), dim3(kBlock), 0, s, n, in, (float*)c0, (float*)c1);
  return hipGetLastError();
}

hipError_t launch_sub_scalar(int64_t count, const double* in, double* out, const double* sub, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_scalar, dim3(blocks_for(count, kBlock)), dim3(kBlock), 0, s, count, in, out, sub);
  return hipGetLastError();
}

hipError_t launch_set_ctl_open(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_set_open, dim3(1), dim3(1), 0, s, ctl);
  return hipGetLastError();
}

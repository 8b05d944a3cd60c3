// Particle-side kernels: binning, deterministic bin sort, owner-computes
// charge spread, force/energy gather and the short-range pair term.
#include <algorithm>
#include <type_traits>

#include "kern.h"
#include "launch.h"
#include "pairs.h"

namespace {

constexpr int kBlock = 256;

// Mesh coordinate u = (x/L - floor(x/L)) * N in FP64, then the first stencil
// index and the fractional offset tau in [0,1) with weight j = M_p(tau+p-1-j)
// (even p: nearest p points around u; odd p: centred on the nearest point).
__device__ __forceinline__ void stencil_origin(double x, double box, int n, int p, int* first,
                                               double* tau) {
  double s = x / box;
  s -= floor(s);
  double u = s * n;
  if (p & 1) {
    double f = floor(u + 0.5);
    *first = (int)f - (p - 1) / 2;
    *tau = u + 0.5 - f;
  } else {
    double f = floor(u);
    *first = (int)f - p / 2 + 1;
    *tau = u - f;
  }
  if (*tau >= 1.0) *tau = 0.0, *first += 1;   // u rounded up onto the next knot
  if (*tau < 0.0) *tau = 0.0;
}

// Tile key of every atom (the 8^3 tile holding its first stencil index) and
// its slot in the tile's count; a non-finite coordinate raises the NaN flag.
// Consecutive atoms often share a tile (the sites of a molecule), so each
// run of equal keys among consecutive lanes takes its slots with one atomic
// add by the run's first lane (the order of slots within a tile is free: the
// bin sort orders each tile's atoms by class and index).
struct BinTiles {
  struct Args {
    int n_atoms, n, p, tile, ntx;
    double box;
    const double* pos;
    int *key, *slot, *count;
    Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void BinTiles::run(const Args& A, Grid G) {
  const int n_atoms = A.n_atoms, n = A.n, p = A.p, tile = A.tile, ntx = A.ntx;
  const int a = G.b * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool on = a < n_atoms;
  int k = -1 - lane;   // distinct from every key and from the other lanes' past the end
  if (on) {
    int tk[3];
    for (int d = 0; d < 3; d++) {
      double x = A.pos[3 * a + d];
      if (!isfinite(x)) {
        A.ctl->nan_flag = 1;
        x = 0.0;
      }
      int first;
      double tau;
      stencil_origin(x, A.box, n, p, &first, &tau);
      int f = first % n;
      if (f < 0) f += n;
      tk[d] = f / tile;
    }
    k = (tk[2] * ntx + tk[1]) * ntx + tk[0];
    A.key[a] = k;
  }
  // runs of equal keys: each lane finds its run's first lane (max-scan of
  // the run heads) and the next run's first lane (min-scan from the right)
  const int prev = __shfl_up(k, 1, 64), next = __shfl_down(k, 1, 64);
  const bool head = lane == 0 || prev != k;
  const bool tail = lane == 63 || next != k;
  int first = head ? lane : 0, last = tail ? lane : 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(first, o, 64), v = __shfl_down(last, o, 64);
    if (lane >= o) first = max(first, u);
    if (lane + o < 64) last = min(last, v);
  }
  int base = 0;
  if (head && on) base = atomicAdd(&A.count[k], last - first + 1);
  base = __shfl(base, first, 64);
  if (on) A.slot[a] = base + (lane - first);
}

// Atom records in bin order, written by the bin sort: rb[i] = {stencil
// origin x | y << 10 | z << 20, atom index} and rq[i] = {charge, tau_x,
// tau_y, tau_z} (the fractional offsets the B-spline weights are computed
// from), so the tile kernels read their atoms' 40 bytes coalesced instead of
// gathering them by atom index, and form the weights themselves.
__device__ __forceinline__ int org_pack(int x, int y, int z) { return x | (y << 10) | (z << 20); }
__device__ __forceinline__ int org_x(int o) { return o & 1023; }
__device__ __forceinline__ int org_y(int o) { return (o >> 10) & 1023; }
__device__ __forceinline__ int org_z(int o) { return o >> 20; }

// Stencil origin (wrapped into [0, n)) and fractional offset of atom a.
__device__ __forceinline__ void atom_origin(int a, int n, int p, double box, const double* pos, int f3[3],
                                            double tau3[3]) {
  for (int d = 0; d < 3; d++) {
    double x = pos[3 * a + d];
    if (!isfinite(x)) x = 0.0;
    int first;
    stencil_origin(x, box, n, p, &first, &tau3[d]);
    int f = first % n;
    if (f < 0) f += n;
    f3[d] = f;
  }
}

// Class of an atom within its tile's bin: bit d set when its stencil crosses
// the upper face of the tile along axis d (so it also reaches the next tile
// along d).  A tile's spread needs, from the bin of the tile d below it, only
// the classes that contain every bit of d.
__device__ __forceinline__ int cross_class(const int f3[3], int tile, int p) {
  int c = 0;
  for (int d = 0; d < 3; d++) c |= ((f3[d] % tile) + p - 1 >= tile) << d;
  return c;
}

struct BinCells {
  struct Args {
    int n_atoms, nc;
    double box;
    const double* pos;
    int *key, *slot, *count;
    Ctl* ctl;
    const int* gate;   // non-null: do nothing unless *gate (rebuild of the neighbour list)
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void BinCells::run(const Args& A, Grid G) {
  if (A.gate && !*A.gate) return;
  const int n_atoms = A.n_atoms, nc = A.nc;
  const double box = A.box;
  const double* __restrict__ pos = A.pos;
  int* __restrict__ key = A.key;
  int* __restrict__ slot = A.slot;
  int* __restrict__ count = A.count;
  Ctl* ctl = A.ctl;
  int a = G.b * kBlock + threadIdx.x;
  if (a >= n_atoms) return;
  int c[3];
  for (int d = 0; d < 3; d++) {
    double x = pos[3 * a + d];
    if (!isfinite(x)) {
      ctl->nan_flag = 1;
      x = 0.0;
    }
    double s = x / box;
    s -= floor(s);
    int ci = (int)(s * nc);
    c[d] = ci >= nc ? nc - 1 : ci;
  }
  int k = (c[2] * nc + c[1]) * nc + c[0];
  key[a] = k;
  slot[a] = atomicAdd(&count[k], 1);
}

// Exclusive scan of the bin counts in three passes: per-chunk sums, one
// workgroup scanning the chunk sums, then each chunk rescanned with its
// offset (integers: exact and order-independent).  Counts are zeroed for
// the next binning.
constexpr int kScanPer = 16;                     // counts per thread
constexpr int kScanChunk = kBlock * kScanPer;    // counts per workgroup

struct ScanSums {
  struct Args {
    int nbins;
    const int* count;
    int* bsum;
    const int* gate;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void ScanSums::run(const Args& A, Grid G) {
  if (A.gate && !*A.gate) return;
  const int nbins = A.nbins;
  const int* __restrict__ count = A.count;
  int* __restrict__ bsum = A.bsum;
  __shared__ int sh[kBlock];
  const int base = G.b * kScanChunk + threadIdx.x * kScanPer;
  int s = 0;
  for (int q = 0; q < kScanPer; q++) s += base + q < nbins ? count[base + q] : 0;
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[G.b] = sh[0];
}

struct ScanTop {
  struct Args {
    int nb;
    int* bsum;
    const int* gate;
  };
  static constexpr int kThreads = 1024;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void ScanTop::run(const Args& A, Grid) {
  if (A.gate && !*A.gate) return;
  const int nb = A.nb;
  int* __restrict__ bsum = A.bsum;
  __shared__ int sh[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = t * per, b1 = min(nb, b0 + per);
  int local = 0;
  for (int b = b0; b < b1; b++) local += bsum[b];
  sh[t] = local;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int acc = sh[t] - local;
  for (int b = b0; b < b1; b++) {
    const int v = bsum[b];
    bsum[b] = acc;
    acc += v;
  }
  if (t == 1023) bsum[nb] = sh[1023];
}

struct ScanFill {
  struct Args {
    int nbins, nb;
    int *count, *start;
    const int* bsum;
    const int* gate;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
// With bsum null (one workgroup covers every count) the offsets start at 0
// and the total comes from this workgroup's own scan.
__device__ void ScanFill::run(const Args& A, Grid G) {
  if (A.gate && !*A.gate) return;
  const int nbins = A.nbins, nb = A.nb;
  int* __restrict__ count = A.count;
  int* __restrict__ start = A.start;
  const int* __restrict__ bsum = A.bsum;
  __shared__ int sh[kBlock];
  const int base = G.b * kScanChunk + threadIdx.x * kScanPer;
  int v[kScanPer];
  int s = 0;
  for (int q = 0; q < kScanPer; q++) {
    v[q] = base + q < nbins ? count[base + q] : 0;
    s += v[q];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int u = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += u;
    __syncthreads();
  }
  int acc = (bsum ? bsum[G.b] : 0) + sh[threadIdx.x] - s;
  for (int q = 0; q < kScanPer; q++) {
    if (base + q < nbins) {
      start[base + q] = acc;
      count[base + q] = 0;
    }
    acc += v[q];
  }
  if (G.b == 0 && threadIdx.x == 0) start[nbins] = bsum ? bsum[nb] : sh[kBlock - 1];
}

struct Scatter {
  struct Args {
    int n_atoms;
    const int *key, *slot, *start;
    int* perm_raw;
    const int* gate;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    if (A.gate && !*A.gate) return;
    int a = G.b * kBlock + threadIdx.x;
    if (a >= A.n_atoms) return;
    A.perm_raw[A.start[A.key[a]] + A.slot[a]] = a;
  }
};

// One wave per bin: rank of each entry = number of smaller keys in the bin
// (keys are distinct), so perm[start + rank] is the sorted list.  The key is
// the atom index; for the mesh bins (rb set) it is (class, atom index), the
// sorted entry is not stored, the atom's records are written at its sorted
// position instead (the records described above) and cls[8 b + c] receives
// the first position of class c in bin b.
struct SortBins {
  struct Args {
    int nbins;
    const int *start, *perm_raw;
    int* perm;
    int n_atoms, n, p, tile;
    double box;
    const double *pos, *qa;
    int2* rb;
    double4* rq;
    int* cls;
    const int* gate;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
// One bin, any size, in chunks of 64 entries.
__device__ void sort_one_bin(const SortBins::Args& A, int bin, int lane) {
  const int* __restrict__ start = A.start;
  const int* __restrict__ perm_raw = A.perm_raw;
  const int s0 = start[bin], cnt = start[bin + 1] - s0;
  const bool mesh = A.rb != nullptr;
  // key of entry i: (class << 32) | atom index (class 0 for the cell bins)
  auto key_of = [&](int i, int* f3, double* tau3) -> long long {
    if (i >= cnt) return 0x7fffffffffffffffLL;
    const int a = perm_raw[s0 + i];
    if (!mesh) return a;
    atom_origin(a, A.n, A.p, A.box, A.pos, f3, tau3);
    return ((long long)cross_class(f3, A.tile, A.p) << 32) | (long long)a;
  };
  int ncls[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i0 = 0; i0 < cnt; i0 += 64) {
    const int i = i0 + lane;
    int f3[3];
    double tau3[3];
    // the entry's charge is loaded with its position, ahead of the ranking
    double qi = 0.0;
    if (mesh && i < cnt) qi = A.qa[perm_raw[s0 + i]];
    const long long v = key_of(i, f3, tau3);
    int rank = 0;
    for (int j0 = 0; j0 < cnt; j0 += 64) {
      int g3[3];
      double t3[3];
      const long long vj_own = j0 == i0 ? v : key_of(j0 + lane, g3, t3);
      const int lim = min(64, cnt - j0);
      for (int jj = 0; jj < lim; jj++) {
        const long long vj = __shfl(vj_own, jj, 64);
        rank += (vj < v);
      }
    }
    if (i < cnt) {
      const int a = (int)(v & 0xffffffffLL);
      if (mesh) {
        A.rb[s0 + rank] = make_int2(org_pack(f3[0], f3[1], f3[2]), a);
        A.rq[s0 + rank] = make_double4(qi, tau3[0], tau3[1], tau3[2]);
      } else {
        A.perm[s0 + rank] = a;
      }
    }
    if (mesh)
      for (int c = 0; c < 8; c++) ncls[c] += __popcll(__ballot(i < cnt && (int)(v >> 32) == c));
  }
  if (mesh && lane == 0) {
    int off = s0;
    for (int c = 0; c < 8; c++) {
      A.cls[8 * bin + c] = off;
      off += ncls[c];
    }
  }
}

// Stencil origin (wrapped first index) and fractional offsets of an atom
// from its already loaded coordinates (the steps of atom_origin).
__device__ __forceinline__ void origin_of(const double x3[3], int n, int p, double box, int f3[3], double tau3[3]) {
  for (int d = 0; d < 3; d++) {
    const double x = isfinite(x3[d]) ? x3[d] : 0.0;
    int first;
    stencil_origin(x, box, n, p, &first, &tau3[d]);
    int f = first % n;
    if (f < 0) f += n;
    f3[d] = f;
  }
}

__device__ void SortBins::run(const Args& A, Grid G) {
  if (A.gate && !*A.gate) return;
  const int nbins = A.nbins;
  const int wave = (G.b * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (!A.rb) {   // cell bins: one per wave
    if (wave < nbins) sort_one_bin(A, wave, lane);
    return;
  }
  // Tile bins: two adjacent bins per wave.  The sort of one small bin is a
  // chain of dependent loads (range, entries, positions) with little work
  // between; when both bins fit a wave, the two chains run side by side.
  const int b0 = 2 * wave;
  if (b0 >= nbins) return;
  const bool two = b0 + 1 < nbins;
  const int s0 = A.start[b0], s1 = A.start[b0 + 1], s2 = two ? A.start[b0 + 2] : s1;
  const int c0 = s1 - s0, c1 = s2 - s1;
  if (c0 > 64 || c1 > 64) {
    sort_one_bin(A, b0, lane);
    if (two) sort_one_bin(A, b0 + 1, lane);
    return;
  }
  const int* __restrict__ perm_raw = A.perm_raw;
  const bool in0 = lane < c0, in1 = lane < c1;
  int a0 = 0, a1 = 0;
  if (in0) a0 = perm_raw[s0 + lane];
  if (in1) a1 = perm_raw[s1 + lane];
  double x0[3] = {0.0, 0.0, 0.0}, x1[3] = {0.0, 0.0, 0.0}, q0 = 0.0, q1 = 0.0;
  if (in0) {
    q0 = A.qa[a0];
    for (int d = 0; d < 3; d++) x0[d] = A.pos[3 * a0 + d];
  }
  if (in1) {
    q1 = A.qa[a1];
    for (int d = 0; d < 3; d++) x1[d] = A.pos[3 * a1 + d];
  }
  int f0[3], f1[3];
  double t0[3], t1[3];
  origin_of(x0, A.n, A.p, A.box, f0, t0);
  origin_of(x1, A.n, A.p, A.box, f1, t1);
  constexpr long long kNone = 0x7fffffffffffffffLL;
  const long long v0 = in0 ? ((long long)cross_class(f0, A.tile, A.p) << 32) | (long long)a0 : kNone;
  const long long v1 = in1 ? ((long long)cross_class(f1, A.tile, A.p) << 32) | (long long)a1 : kNone;
  int r0 = 0, r1 = 0;
  for (int jj = 0; jj < max(c0, c1); jj++) {
    const long long u0 = __shfl(v0, jj, 64), u1 = __shfl(v1, jj, 64);
    r0 += (u0 < v0);   // entries past the bin hold kNone: never smaller
    r1 += (u1 < v1);
  }
  if (in0) {
    A.rb[s0 + r0] = make_int2(org_pack(f0[0], f0[1], f0[2]), a0);
    A.rq[s0 + r0] = make_double4(q0, t0[0], t0[1], t0[2]);
  }
  if (in1) {
    A.rb[s1 + r1] = make_int2(org_pack(f1[0], f1[1], f1[2]), a1);
    A.rq[s1 + r1] = make_double4(q1, t1[0], t1[1], t1[2]);
  }
  int off0 = s0, off1 = s1;
  for (int c = 0; c < 8; c++) {
    const int k0 = __popcll(__ballot(in0 && (int)(v0 >> 32) == c));
    const int k1 = __popcll(__ballot(in1 && (int)(v1 >> 32) == c));
    if (lane == 0) {
      A.cls[8 * b0 + c] = off0;
      if (two) A.cls[8 * b0 + 8 + c] = off1;
    }
    off0 += k0;
    off1 += k1;
  }
}

// Owner-computes spread.  The mesh is cut into TS^3 tiles; atoms are keyed
// by the tile holding their first stencil index (p <= TS, so a stencil
// reaches at most the next tile along each axis).  The atoms that reach a
// tile are those of its own bin and, from the bin of the tile d below it
// (d in {0,1}^3), those whose class (the faces their stencil crosses)
// contains d: at most 27 contiguous ranges of class-sorted bins.
//
// One wave per tile, one lane per 2x2x2 block of it, the block's eight
// values held in registers.  The tile's candidate atoms are staged in the
// wave's part of LDS in chunks of 64 (ranges, then positions), one atom per
// lane, which also forms the atom's B-spline weights laid out over the
// tile: q w_x at the TS x-positions, w_y and w_z likewise, zero where the
// stencil does not reach; the lanes then walk the staged atoms in order and
// every lane adds the atom's terms ((q w_x) w_y) w_z to its block, reading
// its own pair of entries along each axis (exact zeros outside the atom's
// reach, so the walk has no branches and no index arithmetic).  A block per
// lane instead of a column cuts the LDS bytes a lane reads per atom from
// 10 to 6 values (the walk is bound by LDS, the z weights being read by
// every lane).  Each mesh value is a sum in a fixed order (the candidates' order)
// formed in one register: no atomics of any kind, bitwise reproducible, and
// the tile is written once.  The next chunk's records are loaded while the
// current chunk is walked.  TO is the stored precision of q and the
// precision of the sums: FP64, or FP32 for the FP32 charge source (the
// weights are formed in FP64 and rounded once; the fixed order keeps the
// FP32 sums reproducible).
template <typename TO, int TS, int P>
struct Spread {
  using T = TO;   // weights and column sums in the stored precision
  struct Args {
    int n, ntx;
    double box;
    const int *start, *cls;
    const int2* rb;
    const double4* rq;
    TO* q;
  };
  static constexpr int kThreads = kBlock;   // four waves, four tiles
  static constexpr int kChunk = 64;         // staged atoms per round (one per lane)
  __device__ static void run(const Args& A, Grid G);
};
template <typename TO, int TS, int P>
__device__ void Spread<TO, TS, P>::run(const Args& A, Grid G) {
  static_assert(TS == 8, "one lane per 2x2x2 block of the tile");
  // per atom: q w_x, w_y and w_z each laid out over the tile's TS positions
  // along its axis (zero where the stencil does not reach)
  constexpr int NW = kBlock / 64, CH = kChunk, WPA = 3 * TS;
  const int n = A.n, ntx = A.ntx;
  const int* __restrict__ start = A.start;
  const int* __restrict__ cls = A.cls;
  const int2* __restrict__ rb = A.rb;
  const double4* __restrict__ rq = A.rq;
  TO* __restrict__ q = A.q;
  __shared__ __align__(16) T sw[NW][CH * WPA];
  __shared__ int r_lo[NW][64], r_off[NW][65];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ntiles = ntx * ntx * ntx;
  const int t = G.b * NW + wv;
  if (t >= ntiles) return;   // per wave: the kernel has no workgroup barriers
  const int tx = t % ntx, ty = (t / ntx) % ntx, tz = t / (ntx * ntx);
  const int ox = tx * TS, oy = ty * TS, oz = tz * TS;
  // this lane's 2x2x2 block of the tile: x = 2 xp + {0, 1}, y = 2 yp + {0,
  // 1}, z = 2 zp + {0, 1}
  const int xp = lane & 3, yp = (lane >> 2) & 3, zp = lane >> 4;
  // the ranges: lane k = (d, c), d = k >> 3 the lower neighbour, c = k & 7
  // the class; used when c contains d (all classes of the tile's own bin;
  // with one tile per axis, only the own bin)
  int tot;
  {
    const int nd = ntx > 1 ? 2 : 1;
    const int d = lane >> 3, c = lane & 7;
    const int dx = d & 1, dy = (d >> 1) & 1, dz = d >> 2;
    int lo = 0, len = 0;
    if ((c & d) == d && dx < nd && dy < nd && dz < nd) {
      int sx = tx - dx, sy = ty - dy, sz = tz - dz;
      sx += sx < 0 ? ntx : 0;
      sy += sy < 0 ? ntx : 0;
      sz += sz < 0 ? ntx : 0;
      const int b = (sz * ntx + sy) * ntx + sx;
      lo = cls[8 * b + c];
      len = (c < 7 ? cls[8 * b + c + 1] : start[b + 1]) - lo;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o, 64);
      incl += lane >= o ? u : 0;
    }
    r_lo[wv][lane] = lo;
    r_off[wv][lane + 1] = incl;
    if (lane == 0) r_off[wv][0] = 0;
    tot = __shfl(incl, 63, 64);
  }
  int2 nr = make_int2(0, 0);
  double4 nq = make_double4(0.0, 0.0, 0.0, 0.0);
  auto fetch = [&](int c0) {
    if (lane < min(CH, tot - c0)) {
      const int c = c0 + lane;
      int lo = 0, hi = 63;   // last range whose offset is <= c
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (r_off[wv][mid] <= c) lo = mid;
        else hi = mid - 1;
      }
      const int ps = r_lo[wv][lo] + (c - r_off[wv][lo]);   // position in bin order
      nr = rb[ps];
      nq = rq[ps];
    }
  };
  T acc[2][2][2];   // [x][y][z] within the lane's block
#pragma unroll
  for (int u = 0; u < 8; u++) acc[u >> 2][(u >> 1) & 1][u & 1] = T(0);
  fetch(0);
  T* const wsw = sw[wv];
  for (int c0 = 0; c0 < tot; c0 += CH) {
    const int m = __builtin_amdgcn_readfirstlane(min(CH, tot - c0));
    if (lane < m) {
      const double tau3[3] = {nq.y, nq.z, nq.w};
      const int b3[3] = {org_x(nr.x), org_y(nr.x), org_z(nr.x)}, o3[3] = {ox, oy, oz};
      T* wi = wsw + lane * WPA;
      for (int d = 0; d < 3; d++) {
        double wl[P];
        bspline_weights<double>(P, tau3[d], wl);
        int rel = b3[d] - o3[d];   // stencil start relative to the tile, mod n
        rel += rel < 0 ? n : 0;
        rel = rel < TS ? rel : rel - n;   // in [-(p-1), TS)
        // zeros over the tile, then the weights at the positions the
        // stencil reaches (this lane's stores land in order)
        T* wd = wi + d * TS;
#pragma unroll
        for (int x = 0; x < TS; x++) wd[x] = T(0);
#pragma unroll
        for (int j = 0; j < P; j++) {
          int x = rel + j;
          if (ntx == 1) x &= n - 1;   // the tile is the whole periodic mesh
          if ((unsigned)x < (unsigned)TS) wd[x] = (T)(d == 0 ? nq.x * wl[j] : wl[j]);
        }
      }
    }
    // the wave's LDS stores precede its loads below (one wave, in order)
    __builtin_amdgcn_wave_barrier();
    if (c0 + CH < tot) fetch(c0 + CH);
    // one staged atom's entries for this lane's block: q w_x at its two x,
    // w_y at its two y and w_z at its two z positions (8-byte aligned pairs)
    using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    auto load_atom = [&](int j, V2* a, V2* b, V2* c) {
      const T* wj = wsw + j * WPA;
      *a = *reinterpret_cast<const V2*>(wj + 2 * xp);
      *b = *reinterpret_cast<const V2*>(wj + TS + 2 * yp);
      *c = *reinterpret_cast<const V2*>(wj + 2 * TS + 2 * zp);
    };
    // the atom's terms ((q w_x) w_y) w_z at the block's eight points
    auto add_atom = [&](const V2& a, const V2& b, const V2& c) {
      const T ax[2] = {a.x, a.y}, by[2] = {b.x, b.y}, cz[2] = {c.x, c.y};
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int k = 0; k < 2; k++) {
          const T txy = ax[i] * by[k];
#pragma unroll
          for (int l = 0; l < 2; l++) acc[i][k][l] += txy * cz[l];
        }
    };
    int j = 0;
    for (; j + 1 < m; j += 2) {   // two atoms' loads in flight, added in order
      V2 a[2], b[2], c[2];
      load_atom(j, &a[0], &b[0], &c[0]);
      load_atom(j + 1, &a[1], &b[1], &c[1]);
      add_atom(a[0], b[0], c[0]);
      add_atom(a[1], b[1], c[1]);
    }
    if (j < m) {
      V2 a, b, c;
      load_atom(j, &a, &b, &c);
      add_atom(a, b, c);
    }
    __builtin_amdgcn_wave_barrier();
  }
  // two consecutive x values per store (ox + 2 xp is even)
  using O2 = typename std::conditional<sizeof(TO) == 4, float2, double2>::type;
#pragma unroll
  for (int k = 0; k < 2; k++)
#pragma unroll
    for (int l = 0; l < 2; l++) {
      O2 v;
      v.x = (TO)acc[0][k][l];
      v.y = (TO)acc[1][k][l];
      *reinterpret_cast<O2*>(q + nat_idx(n, ox + 2 * xp, oy + 2 * yp + k, oz + 2 * zp + l)) = v;
    }
}

// Gather: F = -k Q sum_n W(r - r_n) (D phi)_n with the central difference D,
// rewritten as derivative weights on a (p+2)^3 neighbourhood, and the
// per-atom energy 1/2 k Q (W * phi)(r).  Sums over a z-plane of the
// neighbourhood in precision T (the weights are rounded to T), the plane's z
// weight and the sum over planes in FP64.
//
// A capped grid of workgroups walks the TS^3 tiles (the spread's bins).  For
// each tile the potential on the tile plus its (p+1)-point halo is staged in
// LDS once; the tile's atoms (its bin, sorted) are then evaluated from LDS,
// one thread per (atom, z-plane of the neighbourhood); the plane partial sums
// are added in a fixed order.
// HO = 1 takes the fourth-order gradient (8 (f_{+1} - f_{-1}) - (f_{+2} -
// f_{-2})) / 12h of the Mehrstellen discretisation instead, on a (p+4)^3
// neighbourhood.
template <typename T, typename TP, int TS, int P, int HO>
struct Gather {
  struct Args {
    int n_atoms, n, p, ntx;
    double h, k_e;
    const int* start;
    const int2* rb;
    const double4* rq;
    const TP *phi0, *phi1;
    double *force, *partial;
    const Ctl* ctl;
    const Ctl* gate;   // non-null: do nothing unless gate->done (solve converged)
  };
  static constexpr int kThreads = kBlock;
  // occupancy floor where the registers allow it (p = 5 second order: five
  // workgroups per CU in FP32, three in FP64)
  static constexpr int kWavesPerEu = ((P <= 5 && HO == 0) || P <= 4) ? (sizeof(T) == 4 ? 5 : 3) : 1;
  static constexpr int GR = 1 + HO;          // reach of the difference
  static constexpr int E = TS + P - 1 + 2 * GR;   // halo tile edge
  static constexpr int PE = P + 2 * GR;      // neighbourhood edge (stencil plus the difference)
  __device__ static void run(const Args& A, Grid G);
};
template <typename T, typename TP, int TS, int P, int HO>
__device__ void Gather<T, TP, TS, P, HO>::run(const Args& A, Grid G) {
  static_assert(E * E <= kBlock, "one halo column per thread");
  const int n = A.n, ntx = A.ntx;
  const double h = A.h, k_e = A.k_e;
  const int* __restrict__ start = A.start;
  const int2* __restrict__ rb = A.rb;
  const double4* __restrict__ rq = A.rq;
  double* __restrict__ force = A.force;
  double* __restrict__ partial = A.partial;
  const Ctl* ctl = A.ctl;
  if (A.gate && !A.gate->done) return;
  __shared__ T sphi[E * E * E];
  __shared__ double part[kBlock][4];
  __shared__ double sh[kBlock / 64];
  constexpr int kSW = 128;            // atoms of a tile whose weights are formed once, while the halo is staged
  static_assert(kSW <= kBlock, "one thread per staged atom record");
  __shared__ T sw[kSW][3][P];
  // the new potential: written over phi^k on a cold solve, over phi^{k-1} otherwise
  const TP* __restrict__ phi = (ctl->cold ? ctl->k_idx : 1 - ctl->k_idx) ? A.phi1 : A.phi0;
  constexpr int per_round = kBlock / PE;   // atoms evaluated per round
  const T inv2h = (T)(0.5 / h);
  const T inv12h = (T)(1.0 / (12.0 * h));
  const int tid = threadIdx.x;
  double e_sum = 0.0;
  const int ntiles = ntx * ntx * ntx;
  // ntx = n / 8 is a power of two: tile coordinates by shifts and masks
  const int lt = __builtin_ctz(ntx), tm = ntx - 1;
  // Everything a tile starts with is loaded into registers while the
  // previous tile is evaluated: its halo column (this thread's (x, y)
  // position, all z), the fractional offset of this thread's (atom,
  // dimension) weight task, and atom tid's origin, index and charge.  Their
  // addresses need the tile's atom range, which is loaded one tile further
  // ahead.  The staging phase moves them into LDS (weights, records), so the
  // rounds use no register whose load may still be in flight: the compiler
  // cannot follow such a load round the loop and waits for every load there,
  // the next tile's halo included.
  TP hv[E];
  double tw = 0.0;                       // weight task tid: atom tid / 3, dimension tid % 3
  int p_org = 0, p_ka = 0;               // atom tid: stencil origin, atom index
  double p_q = 0.0;                      // atom tid: charge
  int cur_lo = 0, cur_hi = 0;            // atom range of the tile being prefetched
  // the tile after it: lane 0 holds its start, lane 1 its end (a vector
  // load: a scalar load would be waited for at the next barrier)
  int nxt = 0;
  __shared__ int s_org[kSW], s_ka[kSW];
  __shared__ double s_q[kSW];
  auto fetch = [&](int t) {
    const int tx = t & tm, ty = (t >> lt) & tm, tz = t >> (2 * lt);
    const int ox = tx * TS - GR, oy = ty * TS - GR, oz = tz * TS - GR;   // halo origin
    if (tid < E * E) {
      const int lx = tid % E, ly = tid / E;
      const TP* col = phi + (size_t)((oy + ly) & (n - 1)) * n + ((ox + lx) & (n - 1));
#pragma unroll
      for (int lz = 0; lz < E; lz++) hv[lz] = col[(size_t)((oz + lz) & (n - 1)) * n * n];
    }
    const int na = cur_hi - cur_lo;
    if (tid < 3 * min(na, kSW)) {
      const int ai = tid / 3, d = tid - 3 * ai;
      tw = reinterpret_cast<const double*>(rq + cur_lo + ai)[1 + d];
    }
    if (tid < min(na, kSW)) {
      const int2 r = rb[cur_lo + tid];
      p_org = r.x;
      p_ka = r.y;
      p_q = rq[cur_lo + tid].x;
    }
  };
  if (G.b < ntiles) {
    cur_lo = start[G.b];
    cur_hi = start[G.b + 1];
    fetch(G.b);
    if (G.b + G.g < ntiles) nxt = start[G.b + G.g + (tid & 1)];
  }
  for (int t = G.b; t < ntiles; t += G.g) {
    const int tx = t & tm, ty = (t >> lt) & tm, tz = t >> (2 * lt);
    const int ox = tx * TS - GR, oy = ty * TS - GR, oz = tz * TS - GR;   // halo origin
    const int a0 = cur_lo, na_t = cur_hi - cur_lo;
    __syncthreads();   // the previous tile's LDS reads are done
    if (tid < E * E) {
#pragma unroll
      for (int lz = 0; lz < E; lz++) sphi[lz * E * E + tid] = (T)hv[lz];
    }
    if (tid < min(na_t, kSW)) {
      s_org[tid] = p_org;
      s_ka[tid] = p_ka;
      s_q[tid] = p_q;
    }
    // each atom's weights, one (atom, dimension) per thread, formed once
    // instead of by each of the atom's plane threads (tasks past the first
    // kBlock, in tiles of more than kBlock / 3 atoms, load their offset here)
    for (int u = tid; u < 3 * min(na_t, kSW); u += kBlock) {
      const int ai = u / 3, d = u - 3 * ai;
      const double x = u == tid ? tw : reinterpret_cast<const double*>(rq + a0 + ai)[1 + d];
      double wl[P];
      bspline_weights<double>(P, x, wl);
#pragma unroll
      for (int j = 0; j < P; j++) sw[ai][d][j] = (T)wl[j];
    }
    if (t + G.g < ntiles) {
      cur_lo = __builtin_amdgcn_readlane(nxt, 0);
      cur_hi = __builtin_amdgcn_readlane(nxt, 1);
      fetch(t + G.g);
      if (t + 2 * G.g < ntiles) nxt = start[t + 2 * G.g + (tid & 1)];
    }
    __syncthreads();
    // the tile's atoms in chunks of kSW staged records and weights; a chunk
    // after the first (tiles of more than kSW atoms) is staged here, from
    // memory
    for (int c0 = 0; c0 < na_t; c0 += kSW) {
      const int nc = min(kSW, na_t - c0);
      if (c0 > 0) {
        __syncthreads();   // the previous chunk's LDS reads are done
        if (tid < nc) {
          const int ps = a0 + c0 + tid;
          const int2 r = rb[ps];
          s_org[tid] = r.x;
          s_ka[tid] = r.y;
          s_q[tid] = rq[ps].x;
        }
        for (int u = tid; u < 3 * nc; u += kBlock) {
          const int ai = u / 3, d = u - 3 * ai;
          double wl[P];
          bspline_weights<double>(P, reinterpret_cast<const double*>(rq + a0 + c0 + ai)[1 + d], wl);
#pragma unroll
          for (int j = 0; j < P; j++) sw[ai][d][j] = (T)wl[j];
        }
        __syncthreads();
      }
      for (int ag = 0; ag < nc; ag += per_round) {
        const int ai = ag + tid / PE, c = tid % PE;
        if (tid < per_round * PE && ai < nc) {
          T rwx[P], rwy[P], rwz[P];
#pragma unroll
          for (int j = 0; j < P; j++) {
            rwx[j] = sw[ai][0][j];
            rwy[j] = sw[ai][1][j];
            rwz[j] = sw[ai][2][j];
          }
          const int rorg = s_org[ai];
          // extended index j <-> stencil offset j - GR; the derivative weight of
          // point j: d[j] = (w[j-1] - w[j+1]) / 2h, or for the fourth-order
          // difference (8 (w[j-1] - w[j+1]) - (w[j-2] - w[j+2])) / 12h
          T wx[PE], wy[PE], dx[PE], dy[PE], wz[PE];
#pragma unroll
          for (int j = 0; j < PE; j++) {
            wx[j] = (j >= GR && j < GR + P) ? rwx[j - GR] : T(0);
            wy[j] = (j >= GR && j < GR + P) ? rwy[j - GR] : T(0);
            wz[j] = (j >= GR && j < GR + P) ? rwz[j - GR] : T(0);
          }
          auto dif = [&](const T* w, int j) -> T {
            const T lo = j >= 1 ? w[j - 1] : T(0), hi = j + 1 < PE ? w[j + 1] : T(0);
            if constexpr (HO == 0) {
              return (lo - hi) * inv2h;
            } else {
              const T lo2 = j >= 2 ? w[j - 2] : T(0), hi2 = j + 2 < PE ? w[j + 2] : T(0);
              return (T(8) * (lo - hi) - (lo2 - hi2)) * inv12h;
            }
          };
#pragma unroll
          for (int j = 0; j < PE; j++) {
            dx[j] = dif(wx, j);
            dy[j] = dif(wy, j);
          }
          T wz_c = T(0), dz_c = T(0);
#pragma unroll
          for (int j = 0; j < PE; j++)
            if (j == c) {
              wz_c = wz[j];
              dz_c = dif(wz, j);
            }
          // neighbourhood origin in the halo tile: base - GR - (tile origin - GR)
          const int lx0 = org_x(rorg) - (ox + GR), ly0 = org_y(rorg) - (oy + GR), lz0 = org_z(rorg) - (oz + GR);
          // the plane's sums: gx = sum_b w_y[b] (d_x . row b), gy = sum_b
          // d_y[b] (w_x . row b), g0 = sum_b w_y[b] (w_x . row b); the
          // plane's z factor is applied once, in FP64
          T gx = T(0), gy = T(0), g0 = T(0);
          const T* plane = sphi + (lz0 + c) * E * E;
#pragma unroll
          for (int b = 0; b < PE; b++) {
            const T* row = plane + (ly0 + b) * E + lx0;
            T sx = T(0), s0 = T(0);
#pragma unroll
            for (int j = 0; j < PE; j++) {
              const T v = row[j];
              sx += dx[j] * v;
              s0 += wx[j] * v;
            }
            gx += wy[b] * sx;
            gy += dy[b] * s0;
            g0 += wy[b] * s0;
          }
          part[tid][0] = (double)wz_c * (double)gx;
          part[tid][1] = (double)wz_c * (double)gy;
          part[tid][2] = (double)dz_c * (double)g0;
          part[tid][3] = (double)wz_c * (double)g0;
        }
        __syncthreads();
        if (tid < per_round && ag + tid < nc) {
          double fx = 0, fy = 0, fz = 0, pot = 0;
          for (int cc = 0; cc < PE; cc++) {
            fx += part[tid * PE + cc][0];
            fy += part[tid * PE + cc][1];
            fz += part[tid * PE + cc][2];
            pot += part[tid * PE + cc][3];
          }
          const int ka = s_ka[ag + tid];
          const double kqe = k_e * s_q[ag + tid];
          if (force) {
            force[3 * ka] = -kqe * fx;
            force[3 * ka + 1] = -kqe * fy;
            force[3 * ka + 2] = -kqe * fz;
          }
          e_sum += 0.5 * kqe * pot;
        }
        __syncthreads();
      }
    }
  }
  double bs = block_sum(e_sum, sh);
  if (threadIdx.x == 0) partial[G.b] = bs;
}

// One workgroup: *dst = sum of the nb partials (fixed order).
struct FinSum {
  struct Args {
    int nb;
    const double* partial;
    double* dst;
    const Ctl* gate;   // non-null: do nothing unless gate->done
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid) {
    if (A.gate && !A.gate->done) return;
    __shared__ double sh[kBlock / 64];
    const double tot = reduce_partials_sum(A.partial, A.nb, sh);
    if (threadIdx.x == 0) *A.dst = tot;
  }
};

// One workgroup: E_sr and the energy assembly {E_sr, E_lr, E_self, E_total}.
struct FinEnergy {
  struct Args {
    int nb;
    double e_self;
    const double* partial;
    const double* nfpart;   // 3 per workgroup of the pair kernels
    int has_force;          // 0: no force output this step (net force unknown)
    Ctl* ctl;
    double* energy_out;
    int nbr;   // 1: the step used neighbour lists; a flagged rebuild is now done
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid);
};
__device__ void FinEnergy::run(const Args& A, Grid) {
  Ctl* ctl = A.ctl;
  const double e_self = A.e_self;
  double* energy_out = A.energy_out;
  __shared__ double sh[kBlock / 64];
  const double tot = reduce_partials_sum(A.partial, A.nb, sh);
  double nf[3];
  for (int c = 0; c < 3; c++) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < A.nb; i += blockDim.x) acc += A.nfpart[3 * i + c];
    nf[c] = block_sum(acc, sh);
  }
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; c++) ctl->net_force[c] = A.has_force ? nf[c] : __builtin_nan("");
    if (A.nbr && ctl->nbr_stale) {
      ctl->nbr_builds++;
      ctl->nbr_stale = 0;
    }
    ctl->e_sr = tot;
    if (energy_out) {
      energy_out[0] = tot;
      energy_out[1] = ctl->e_lr;
      energy_out[2] = e_self;
      energy_out[3] = tot + ctl->e_lr + e_self;
    }
  }
}

// Cell-ordered packed copy of the atoms, {x, y, z, q} per entry, for the
// pair kernels' coalesced candidate loads.
struct CellPack {
  struct Args {
    int n_atoms;
    const int* cperm;
    const double *pos, *qa;
    double4* spos;
    const int* gate;   // non-null: do nothing unless *gate
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    if (A.gate && !*A.gate) return;
    const int jj = G.b * kBlock + threadIdx.x;
    if (jj >= A.n_atoms) return;
    const int a = A.cperm[jj];
    A.spos[jj] = make_double4(A.pos[3 * a], A.pos[3 * a + 1], A.pos[3 * a + 2], A.qa[a]);
  }
};

// Verlet neighbour list with a skin (Verlet's buffered list): the list of
// the atom at cell-order position wi holds every other atom within
// r_l = r_cut + skin at the last build.  While no atom has moved more than
// skin/2 (minimum image) since then, every pair within r_cut is in it, so
// the pair sums over the list equal those over the cell neighbourhood.
//
// Every step: refresh the cell-ordered copy in the build's order and flag a
// rebuild when some atom has moved too far (a non-finite position, or the
// NaN reference positions of a list never built, also flag it).
struct NbrCheck {
  struct Args {
    int n_atoms;
    double box, half_skin2;
    const int* cperm;
    const double *pos, *qa;
    double4* spos;
    const double4* ref;
    Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    const int jj = G.b * kBlock + threadIdx.x;
    if (jj >= A.n_atoms) return;
    const int a = A.cperm[jj];
    const double x = A.pos[3 * a], y = A.pos[3 * a + 1], z = A.pos[3 * a + 2];
    A.spos[jj] = make_double4(x, y, z, A.qa[a]);
    const double4 r = A.ref[jj];
    const double inv_box = 1.0 / A.box;
    const double dx = min_img(x - r.x, A.box, inv_box), dy = min_img(y - r.y, A.box, inv_box),
                 dz = min_img(z - r.z, A.box, inv_box);
    if (!(dx * dx + dy * dy + dz * dz <= A.half_skin2)) A.ctl->nbr_stale = 1;
  }
};

// The list build (only when flagged), on cells at least r_l wide.  Entries
// are cell-order positions jj in candidate order (the 27-cell neighbourhood
// in the order of candidate_range), so the sums over a list are
// deterministic, with two flag bits: kNbrSameGroup (an exclusion-group partner) and kNbrSite (atom index
// divisible by 3: the O of an O,H,H triple).  Entries past the capacity are
// dropped and the count keeps the true number: such an atom's pair kernels
// fall back to the cell scan.
struct NbrArgs {
  int n_atoms, nc, excl_group, cap;
  double box, rl2;
  const int *cstart, *cperm;
  const double4* spos;
  double4* ref;
  int *list, *cnt;
  Ctl* ctl;
};

// One wave per atom: lanes test 64 consecutive candidates at a time.  Every
// atom loads its whole neighbourhood, so this suits small systems (few
// cells, where a wave per cell would leave the chip idle).
struct NbrBuildAtom {
  using Args = NbrArgs;
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void NbrBuildAtom::run(const Args& A, Grid G) {
  if (!A.ctl->nbr_stale) return;
  const int n_atoms = A.n_atoms, nc = A.nc, g = A.excl_group, cap = A.cap;
  const double box = A.box, rl2 = A.rl2, inv_box = 1.0 / box;
  const int* __restrict__ cstart = A.cstart;
  const int* __restrict__ cperm = A.cperm;
  const double4* __restrict__ spos = A.spos;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int nwaves = G.g * (kBlock / 64);
  for (int wave = (G.b * kBlock + threadIdx.x) >> 6; wave < n_atoms; wave += nwaves) {
    const double4 me = spos[wave];
    const int i = cperm[wave];
    const int gi = g > 0 ? i / g : -1;
    int* __restrict__ out = A.list + (size_t)wave * cap;
    int c[3];
    cell_of(me.x, me.y, me.z, box, nc, c);
    int count = 0;
    int lo = 0, hi = 0;
    for (int r = 0; candidate_range(r, c, nc, cstart, &lo, &hi); r++) {
      for (int b0 = lo; b0 < hi; b0 += 64) {
        const int jj = b0 + lane;
        bool ok = false;
        unsigned e = 0;
        if (jj < hi && jj != wave) {
          const double4 a = spos[jj];
          const double dx = min_img(me.x - a.x, box, inv_box), dy = min_img(me.y - a.y, box, inv_box),
                       dz = min_img(me.z - a.z, box, inv_box);
          if (dx * dx + dy * dy + dz * dz < rl2) {
            const int j = cperm[jj];
            ok = true;
            e = (unsigned)jj | (gi >= 0 && j / g == gi ? kNbrSameGroup : 0u) | (j % 3 == 0 ? kNbrSite : 0u);
          }
        }
        const unsigned long long m = __ballot(ok);
        if (ok) {
          const int slot = count + __popcll(m & below);
          if (slot < cap) out[slot] = (int)e;
        }
        count += __popcll(m);
      }
    }
    if (lane == 0) {
      A.cnt[wave] = count;
      A.ref[wave] = me;
      if (count > cap) atomicAdd(&A.ctl->nbr_over, 1);
    }
  }
}

// One single-wave workgroup per cell: a lane per atom of the cell (64 at a
// time), the candidates of the cell's neighbourhood streamed through LDS 64
// at a time and tested by every lane against its atom, so each candidate is
// loaded once per 64 atoms instead of once per atom.
struct NbrBuildCell {
  using Args = NbrArgs;
  static constexpr int kThreads = 64;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void NbrBuildCell::run(const Args& A, Grid G) {
  if (!A.ctl->nbr_stale) return;
  const int nc = A.nc, g = A.excl_group, cap = A.cap, ncells = nc * nc * nc;
  const double box = A.box, rl2 = A.rl2, inv_box = 1.0 / box;
  const int* __restrict__ cstart = A.cstart;
  const int* __restrict__ cperm = A.cperm;
  const double4* __restrict__ spos = A.spos;
  __shared__ double4 cand[64];
  __shared__ int cidx[64];
  const int lane = threadIdx.x;
  for (int cell = G.b; cell < ncells; cell += G.g) {
    const int c[3] = {cell % nc, (cell / nc) % nc, cell / (nc * nc)};
    const int s0 = cstart[cell], s1 = cstart[cell + 1];
    for (int b = s0; b < s1; b += 64) {
      const int wi = b + lane;
      const bool act = wi < s1;
      const double4 me = act ? spos[wi] : make_double4(0.0, 0.0, 0.0, 0.0);
      const int i = act ? cperm[wi] : 0;
      const int gi = g > 0 ? i / g : -1;
      int* __restrict__ out = A.list + (size_t)(act ? wi : 0) * cap;
      int count = 0;
      int lo = 0, hi = 0;
      for (int r = 0; candidate_range(r, c, nc, cstart, &lo, &hi); r++) {
        for (int c0 = lo; c0 < hi; c0 += 64) {
          const int m = min(64, hi - c0);
          if (lane < m) {
            cand[lane] = spos[c0 + lane];
            cidx[lane] = cperm[c0 + lane];
          }
          wave_sync_lds();
          if (act) {
            for (int t = 0; t < m; t++) {
              const double4 a = cand[t];
              const double dx = min_img(me.x - a.x, box, inv_box), dy = min_img(me.y - a.y, box, inv_box),
                           dz = min_img(me.z - a.z, box, inv_box);
              const int jj = c0 + t;
              if (dx * dx + dy * dy + dz * dz < rl2 && jj != wi) {
                const int j = cidx[t];
                const unsigned e =
                    (unsigned)jj | (gi >= 0 && j / g == gi ? kNbrSameGroup : 0u) | (j % 3 == 0 ? kNbrSite : 0u);
                if (count < cap) out[count] = (int)e;
                count++;
              }
            }
          }
          wave_sync_lds();
        }
      }
      if (act) {
        A.cnt[wi] = count;
        A.ref[wi] = me;
        if (count > cap) atomicAdd(&A.ctl->nbr_over, 1);
      }
    }
  }
}

// Short-range pairs (Eq. 20 force, Eq. 6 energy) with the minimum image;
// pairs inside one exclusion group instead get the Ewald exclusion
// correction -k Q Q erf(alpha r)/r.  One wave per atom; a fixed shuffle tree
// adds the lane sums (deterministic).  force += F_sr.
// LIST: over each atom's neighbour list (atoms over the list capacity are
// skipped); otherwise the cell scan, for every atom (no lists, span 1: one
// atom per wave) or for the atoms over capacity (span 64: each wave picks
// them from 64 consecutive positions by ballot).
// NE = 1 (MD steps on neighbour lists): the same pass over the list also
// adds the non-electrostatic pair term (model 1: Born-Mayer repulsion
// between all pairs; model 2: O-O Lennard-Jones), each shifted to zero at
// r_cut, with its energy in nepart.
template <bool LIST, int NE = 0>
struct ShortRange {
  struct Args {
    int n_atoms, nc, excl_group, span;
    double box, alpha, rc2, k_e;
    const double *pos, *qa;
    const int *cstart, *cperm;
    const double4* spos;   // cell-ordered {x, y, z, q}
    double *force, *partial;
    double* nfpart;           // 3 per workgroup: sum of the atoms' final forces (net force)
    const double* erfc_tab;   // erfcx table on [0, alpha r_cut] (1..kErfcMaxIntervals intervals)
    int erfc_n;
    double erfc_scale;        // table intervals per unit of alpha r
    // neighbour lists (null: none): entries of cell-order atom wi at
    // list + wi * cap, nlist[wi] of them
    const int *list, *nlist;
    int cap;
    // NE: model, parameters (model 1: A, rho; model 2: eps, sigma), energy partials
    int model;
    double ne_p0, ne_p1;
    double* nepart;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};

// The short-range force on the atom at cell-order position `wave` (lanes
// split its pairs, a fixed shuffle tree sums them) and its pair energy,
// accumulated into each lane's en.
template <bool LIST, int NE>
__device__ __forceinline__ void sr_atom(const typename ShortRange<LIST, NE>::Args& A, int wave, const double* tab,
                                        PairQueue* Q, double& en, double* nf, double& ene, double ne_shift) {
  const int n_atoms = A.n_atoms, excl_group = A.excl_group;
  const double box = A.box, alpha = A.alpha, rc2 = A.rc2, k_e = A.k_e;
  const double* __restrict__ pos = A.pos;
  const double* __restrict__ qa = A.qa;
  const int* __restrict__ cperm = A.cperm;
  const double4* __restrict__ spos = A.spos;
  const int tab_n = A.erfc_n;
  const double tab_scale = A.erfc_scale;
  const int lane = threadIdx.x & 63;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const int i = cperm[wave];
  const double4 me = spos[wave];
  const double xi = me.x, yi = me.y, zi = me.z;
  const double qi = me.w;
  const double inv_box = 1.0 / box;
  const double tapi = 2.0 * alpha / sqrt(M_PI);
  const int gi = excl_group > 0 ? i / excl_group : -1;
  // the pair term from r^2 and 1/r (one reciprocal square root serves the
  // erfc term and the non-electrostatic term of the same pair)
  auto pair_ir = [&](double dx, double dy, double dz, double r2, double inv_r, double qj) {
    // erfc(a r) = exp(-a^2 r^2) erfcx(a r), erfcx from the table
    const double r = r2 * inv_r;
    const double x = alpha * r;
    const double g = exp(-x * x);
    const double ec = g * erfcx_table(tab, tab_n, tab_scale, x);
    const double qq = k_e * qi * qj;
    const double f = qq * inv_r * inv_r * (ec * inv_r + tapi * g);
    fx += f * dx; fy += f * dy; fz += f * dz;
    en += 0.5 * qq * ec * inv_r;
  };
  auto pair = [&](double dx, double dy, double dz, double r2, double qj) { pair_ir(dx, dy, dz, r2, rsqrt(r2), qj); };
  if constexpr (LIST && NE != 0) {
    // one pass over the list: the erfc pair and, where it applies, the
    // non-electrostatic pair (model 2: O-O only; the atom is an O when its
    // index is divisible by 3 and the entry's site flag marks an O partner)
    const int model = A.model;
    const double p0 = A.ne_p0, p1 = A.ne_p1, inv_p1 = 1.0 / p1, p1sq = p1 * p1;
    const bool i_site = model == 1 || i % 3 == 0;
    const int* ent = A.list + (size_t)wave * A.cap;
    const int cnt = A.nlist[wave];
    const double inv_b = 1.0 / box;
    for (int k = lane; k < cnt; k += 64) {
      const unsigned e = (unsigned)ent[k];
      const double4 a = spos[e & kNbrIndex];
      const double dx = min_img(xi - a.x, box, inv_b);
      const double dy = min_img(yi - a.y, box, inv_b);
      const double dz = min_img(zi - a.z, box, inv_b);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < rc2)) continue;
      const double inv_r = rsqrt(r2);
      if (!(e & kNbrSameGroup)) pair_ir(dx, dy, dz, r2, inv_r, a.w);
      if (i_site && (model == 1 || (e & kNbrSite))) {
        double f;
        if (model == 1) {
          const double v = p0 * exp(-(r2 * inv_r) * inv_p1);
          f = v * inv_p1 * inv_r;
          ene += 0.5 * (v - ne_shift);
        } else {
          const double inv_r2 = inv_r * inv_r;
          const double sr2 = p1sq * inv_r2;
          const double sr6 = sr2 * sr2 * sr2;
          f = 24.0 * p0 * (2.0 * sr6 * sr6 - sr6) * inv_r2;
          ene += 0.5 * (4.0 * p0 * (sr6 * sr6 - sr6) - ne_shift);
        }
        fx += f * dx; fy += f * dy; fz += f * dz;
      }
    }
  } else if constexpr (LIST)
    for_each_listed(A.list + (size_t)wave * A.cap, A.nlist[wave], xi, yi, zi, box, spos,
                    [&](unsigned e, double r2) { return r2 < rc2 && !(e & kNbrSameGroup); }, pair);
  else
    for_each_pair(wave, xi, yi, zi, box, A.nc, A.cstart, spos, *Q,
                  [&](int jj, double r2) { return r2 < rc2 && !(gi >= 0 && cperm[jj] / excl_group == gi); }, pair);
  if (gi >= 0 && lane < excl_group) {
    const int j = gi * excl_group + lane;
    if (j != i && j < n_atoms) {
      double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
      dx -= box * rint(dx * inv_box);
      dy -= box * rint(dy * inv_box);
      dz -= box * rint(dz * inv_box);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double r = sqrt(r2);
      // erf = 1 - exp(-x^2) erfcx(x); intramolecular pairs lie well inside the table
      const double xr = alpha * r;
      const double er = 1.0 - exp(-xr * xr) * erfcx_table(tab, tab_n, tab_scale, xr);
      const double qq = k_e * qi * qa[j];
      const double f = qq * (tapi * exp(-alpha * alpha * r2) / r - er / r2) / r;
      fx += f * dx; fy += f * dy; fz += f * dz;
      en += -0.5 * qq * er / r;
    }
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  if (lane == 0 && A.force) {
    // the atom's final electrostatic force (the gather wrote the mesh part)
    const double gx = A.force[3 * i] + fx, gy = A.force[3 * i + 1] + fy, gz = A.force[3 * i + 2] + fz;
    A.force[3 * i] = gx;
    A.force[3 * i + 1] = gy;
    A.force[3 * i + 2] = gz;
    nf[0] += gx;
    nf[1] += gy;
    nf[2] += gz;
  }
}

template <bool LIST, int NE>
__device__ void ShortRange<LIST, NE>::run(const Args& A, Grid G) {
  const int n_atoms = A.n_atoms;
  __shared__ double sh[kBlock / 64];
  __shared__ PairQueue queue[LIST ? 1 : kBlock / 64];
  extern __shared__ double tab[];   // erfc_n * (kErfcDeg + 1) coefficients (dynamic LDS)
  __shared__ double shf[3 * (kBlock / 64)];
  const int lane = threadIdx.x & 63;
  const int nwaves = G.g * (kBlock / 64);
  double en = 0.0, ene = 0.0;
  double nf[3] = {0.0, 0.0, 0.0};   // lane 0: net force of the wave's atoms
  double ne_shift = 0.0;            // the non-electrostatic potential at r_cut
  if (NE != 0) {
    if (A.model == 1) {
      ne_shift = A.ne_p0 * exp(-sqrt(A.rc2) / A.ne_p1);
    } else {
      const double s2 = A.ne_p1 * A.ne_p1 / A.rc2, s6 = s2 * s2 * s2;
      ne_shift = 4.0 * A.ne_p0 * (s6 * s6 - s6);
    }
  }
  for (int k = threadIdx.x; k < A.erfc_n * (kErfcDeg + 1); k += kBlock) tab[k] = A.erfc_tab[k];
  __syncthreads();
  if constexpr (LIST) {
    for (int wave = (G.b * kBlock + threadIdx.x) >> 6; wave < n_atoms; wave += nwaves)
      if (A.nlist[wave] <= A.cap) sr_atom<true, NE>(A, wave, tab, nullptr, en, nf, ene, ne_shift);
  } else {
    PairQueue* Q = &queue[threadIdx.x >> 6];
    const int span = A.span;
    for (int chunk = (G.b * kBlock + threadIdx.x) >> 6; chunk * span < n_atoms; chunk += nwaves) {
      const int mine = chunk * span + lane;
      const bool in = lane < span && mine < n_atoms;
      unsigned long long todo = __ballot(in && (!A.list || A.nlist[mine] > A.cap));
      while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;   // wave-uniform
        todo &= todo - 1;
        sr_atom<false, NE>(A, chunk * span + l, tab, Q, en, nf, ene, ne_shift);
      }
    }
  }
  en = wave_sum(en);
  if (NE != 0) ene = wave_sum(ene);
  __shared__ double she[kBlock / 64];
  if (lane == 0) {
    sh[threadIdx.x >> 6] = en;
    if (NE != 0) she[threadIdx.x >> 6] = ene;
    for (int c = 0; c < 3; c++) shf[3 * (threadIdx.x >> 6) + c] = nf[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, se = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < kBlock / 64; k++) {
      s += sh[k];
      if (NE != 0) se += she[k];
      for (int c = 0; c < 3; c++) f[c] += shf[3 * k + c];
    }
    A.partial[G.b] = s;
    if (NE != 0) A.nepart[G.b] = se;
    for (int c = 0; c < 3; c++) A.nfpart[3 * G.b + c] = f[c];
  }
}

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_bin_tiles(int n_atoms, const double* pos, double box, int n, int p, int tile, int ntx, int* key,
                           int* slot, int* count, Ctl* ctl, hipStream_t s) {
  return go<BinTiles>({n_atoms, n, p, tile, ntx, box, pos, key, slot, count, ctl}, blocks_for(n_atoms, kBlock), 0, s);
}

hipError_t launch_bin_cells(int n_atoms, const double* pos, double box, int nc, int* key, int* slot,
                            int* count, Ctl* ctl, hipStream_t s, const int* gate) {
  return go<BinCells>({n_atoms, nc, box, pos, key, slot, count, ctl, gate}, blocks_for(n_atoms, kBlock), 0, s);
}

int scan_partials(int nbins) { return (nbins + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_scan(int nbins, int* count, int* start, int* bsum, hipStream_t s, const int* gate) {
  const int nb = (nbins + kScanChunk - 1) / kScanChunk;
  if (nb == 1) {
    // one workgroup scans all; in a batch recording it takes the sequence
    // position of the multi-workgroup ScanFill, so it merges with the other
    // systems' ScanFill launches
    if (g_recorder) g_recorder->seq += 2;
    return go<ScanFill>({nbins, 1, count, start, nullptr, gate}, 1, 0, s);
  }
  hipError_t e = go<ScanSums>({nbins, count, bsum, gate}, nb, 0, s);
  if (e != hipSuccess) return e;
  e = go<ScanTop>({nb, bsum, gate}, 1, 0, s);
  if (e != hipSuccess) return e;
  return go<ScanFill>({nbins, nb, count, start, bsum, gate}, nb, 0, s);
}

hipError_t launch_scatter(int n_atoms, const int* key, const int* slot, const int* start, int* perm_raw,
                          hipStream_t s, const int* gate) {
  return go<Scatter>({n_atoms, key, slot, start, perm_raw, gate}, blocks_for(n_atoms, kBlock), 0, s);
}

hipError_t launch_sort_bins(int nbins, const int* start, const int* perm_raw, int* perm, Ctl*,
                            hipStream_t s, const int* gate) {
  return go<SortBins>({nbins, start, perm_raw, perm, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr,
                       gate},
                      blocks_for((int64_t)nbins * 64, kBlock), 0, s);
}

hipError_t launch_sort_pack(int nbins, const int* start, const int* perm_raw, int n_atoms, const double* pos,
                            const double* qa, double box, int n, int p, int tile, void* rb, void* rq, int* cls,
                            hipStream_t s) {
  // two tile bins per wave
  return go<SortBins>({nbins, start, perm_raw, nullptr, n_atoms, n, p, tile, box, pos, qa, (int2*)rb, (double4*)rq,
                       cls, nullptr},
                      blocks_for((int64_t)((nbins + 1) / 2) * 64, kBlock), 0, s);
}

namespace {
template <int P>
hipError_t spread_p(bool fp64, int n, int ntx, double box, const int* start, const int* cls, const void* rb,
                    const void* rq, void* q, hipStream_t s) {
  const int ntiles = ntx * ntx * ntx;
  const int grid = (ntiles + 3) / 4;   // one wave per tile
  if (fp64)
    return go<Spread<double, 8, P>>({n, ntx, box, start, cls, (const int2*)rb, (const double4*)rq, (double*)q}, grid,
                                    0, s);
  return go<Spread<float, 8, P>>({n, ntx, box, start, cls, (const int2*)rb, (const double4*)rq, (float*)q}, grid, 0,
                                 s);
}
}  // namespace

hipError_t launch_spread(bool fp64, int n, int p, int tile, int ntx, double box, const int* start, const int* cls,
                         const void* rb, const void* rq, void* q, hipStream_t s) {
  if (tile != 8) return hipErrorInvalidValue;
  switch (p) {
    case 2: return spread_p<2>(fp64, n, ntx, box, start, cls, rb, rq, q, s);
    case 3: return spread_p<3>(fp64, n, ntx, box, start, cls, rb, rq, q, s);
    case 4: return spread_p<4>(fp64, n, ntx, box, start, cls, rb, rq, q, s);
    case 5: return spread_p<5>(fp64, n, ntx, box, start, cls, rb, rq, q, s);
    case 6: return spread_p<6>(fp64, n, ntx, box, start, cls, rb, rq, q, s);
    case 7: return spread_p<7>(fp64, n, ntx, box, start, cls, rb, rq, q, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <int P, int HO>
hipError_t gather_p(bool fp64, int n_atoms, int n, int ntx, double h, double k_e, const int* start, const void* rb,
                    const void* rq, const double* phi0, const double* phi1, const float* phi32, double* force,
                    double* partial, Ctl* ctl, const Ctl* gate, int nb, hipStream_t s) {
  if (fp64)
    return go<Gather<double, double, 8, P, HO>>({n_atoms, n, P, ntx, h, k_e, start, (const int2*)rb, (const double4*)rq,
                                             phi0, phi1, force,
                                             partial, ctl, gate}, nb, 0, s);
  return go<Gather<float, float, 8, P, HO>>({n_atoms, n, P, ntx, h, k_e, start, (const int2*)rb, (const double4*)rq,
                                         phi32, phi32, force,
                                         partial, ctl, gate}, nb, 0, s);
}
}  // namespace

hipError_t launch_gather(bool fp64, int n_atoms, int n, int p, int tile, int ntx, double h, double k_e,
                         const int* start, const void* rb, const void* rq, const double* phi0, const double* phi1,
                         const float* phi32, double* force, double* partial, Ctl* ctl, hipStream_t s, bool finalize,
                         int stencil) {
  if (tile != 8 || (stencil == 1 && p > 5) || ntx < 1 || (ntx & (ntx - 1))) return hipErrorInvalidValue;
  const int nb = std::min(ntx * ntx * ntx, kMaxRedBlocks);
  // the step's gather (finalize) waits for a converged solve
  const Ctl* gate = finalize ? ctl : nullptr;
  hipError_t e;
  switch (p) {
    case 2: e = stencil == 1 ? gather_p<2, 1>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s)
                          : gather_p<2, 0>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s); break;
    case 3: e = stencil == 1 ? gather_p<3, 1>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s)
                          : gather_p<3, 0>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s); break;
    case 4: e = stencil == 1 ? gather_p<4, 1>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s)
                          : gather_p<4, 0>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s); break;
    case 5: e = stencil == 1 ? gather_p<5, 1>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s)
                          : gather_p<5, 0>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s); break;
    case 6: e = gather_p<6, 0>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s); break;
    case 7: e = gather_p<7, 0>(fp64, n_atoms, n, ntx, h, k_e, start, rb, rq, phi0, phi1, phi32, force, partial, ctl, gate, nb, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || !finalize) return e;
  return go<FinSum>({nb, partial, &ctl->e_lr, gate}, 1, 0, s);
}

hipError_t launch_cell_pack(int n_atoms, const int* cperm, const double* pos, const double* qa, void* spos,
                            hipStream_t s, const int* gate) {
  return go<CellPack>({n_atoms, cperm, pos, qa, (double4*)spos, gate}, blocks_for(n_atoms, kBlock), 0, s);
}

hipError_t launch_nbr_check(int n_atoms, double box, double skin, const int* cperm, const double* pos,
                            const double* qa, void* spos, const void* ref, Ctl* ctl, hipStream_t s) {
  const double h = 0.5 * skin;
  return go<NbrCheck>({n_atoms, box, h * h, cperm, pos, qa, (double4*)spos, (const double4*)ref, ctl},
                      blocks_for(n_atoms, kBlock), 0, s);
}

hipError_t launch_nbr_build(int n_atoms, double box, double r_list, int nc, int excl_group, int cap,
                            const int* cstart, const int* cperm, const void* spos, void* ref, int* list, int* nlist,
                            Ctl* ctl, hipStream_t s) {
  if (cap < 1 || (unsigned)(n_atoms - 1) > kNbrIndex) return hipErrorInvalidValue;
  const NbrArgs a{n_atoms, nc, excl_group, cap, box, r_list * r_list, cstart, cperm, (const double4*)spos,
                  (double4*)ref, list, nlist, ctl};
  // a wave per cell once that gives enough waves (each takes its cell's
  // atoms 64 at a time); fewer, fuller cells: a wave per atom
  const int64_t ncells = (int64_t)nc * nc * nc;
  const int64_t per_cell = (n_atoms + ncells - 1) / ncells;
  if (ncells * ((per_cell + 63) / 64) >= 8192)
    return go<NbrBuildCell>(a, (int)std::min<int64_t>(ncells, 65536), 0, s);
  return go<NbrBuildAtom>(a, std::min(blocks_for((int64_t)n_atoms * 64, kBlock), kPartialSlots), 0, s);
}

hipError_t launch_sr(int n_atoms, const double* pos, const double* qa, double box, double alpha,
                     double r_cut, double k_e, int nc, int excl_group, const int* cstart,
                     const int* cperm, const void* spos, const double* erfc_tab, int erfc_n, double erfc_scale,
                     double* force, double e_self, double* energy_out, double* partial, double* nfpart, Ctl* ctl,
                     hipStream_t s, const int* list, const int* nlist, int cap, int ne_model, double ne_p0,
                     double ne_p1, double* nepart, int* ne_written) {
  if (erfc_n < 1 || erfc_n > kErfcMaxIntervals) return hipErrorInvalidValue;
  const size_t lds = (size_t)erfc_n * (kErfcDeg + 1) * sizeof(double);
  const double rc2 = r_cut * r_cut;
  if (ne_written) *ne_written = 0;
  if (!list) {
    const int nb = std::min(blocks_for((int64_t)n_atoms * 64, kBlock), kPartialSlots);
    hipError_t e = go<ShortRange<false>>({n_atoms, nc, excl_group, 1, box, alpha, rc2, k_e, pos, qa, cstart, cperm,
                                          (const double4*)spos, force, partial, nfpart, erfc_tab, erfc_n,
                                          erfc_scale, nullptr, nullptr, 0, 0, 0.0, 0.0, nullptr}, nb, lds, s);
    if (e != hipSuccess) return e;
    return go<FinEnergy>({nb, e_self, partial, nfpart, force != nullptr, ctl, energy_out, 0}, 1, 0, s);
  }
  // the lists (with the non-electrostatic pair term when ne_model != 0),
  // then the cell scan for the atoms over capacity; partials of the first
  // kernel, then of the second
  const int nb = std::min(blocks_for((int64_t)n_atoms * 64, kBlock), kPartialSlots / 2);
  hipError_t e;
  if (ne_model != 0) {
    e = go<ShortRange<true, 1>>({n_atoms, nc, excl_group, 1, box, alpha, rc2, k_e, pos, qa, cstart, cperm,
                                 (const double4*)spos, force, partial, nfpart, erfc_tab, erfc_n, erfc_scale, list,
                                 nlist, cap, ne_model, ne_p0, ne_p1, nepart}, nb, lds, s);
    if (ne_written) *ne_written = nb;
  } else {
    e = go<ShortRange<true>>({n_atoms, nc, excl_group, 1, box, alpha, rc2, k_e, pos, qa, cstart, cperm,
                              (const double4*)spos, force, partial, nfpart, erfc_tab, erfc_n, erfc_scale, list,
                              nlist, cap, 0, 0.0, 0.0, nullptr}, nb, lds, s);
  }
  if (e != hipSuccess) return e;
  const int nb2 = std::min(blocks_for((int64_t)(n_atoms + 63) / 64 * 64, kBlock), kPartialSlots / 2);
  e = go<ShortRange<false>>({n_atoms, nc, excl_group, 64, box, alpha, rc2, k_e, pos, qa, cstart, cperm,
                             (const double4*)spos, force, partial + nb, nfpart + 3 * nb, erfc_tab, erfc_n,
                             erfc_scale, list, nlist, cap, 0, 0.0, 0.0, nullptr}, nb2, lds, s);
  if (e != hipSuccess) return e;
  return go<FinEnergy>({nb + nb2, e_self, partial, nfpart, force != nullptr, ctl, energy_out, 1}, 1, 0, s);
}

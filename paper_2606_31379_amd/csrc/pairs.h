// Neighbour enumeration shared by the pair kernels (one wave per atom).
//
// Atoms are read from a cell-ordered packed copy {x, y, z, q} (built once per
// step after the cell sort), so the candidates of the three cells of one x
// row are one contiguous range (split only where the row wraps around the
// box) and are loaded coalesced.  Each
// lane applies the minimum image and the caller's acceptance test (cutoff,
// exclusions); accepted pairs are appended, in candidate order, to a per-wave
// queue in LDS (ballot + prefix rank), and the pair function -- the
// expensive part, e.g. erfc and exp in FP64 -- runs once per 64 queued pairs
// with every lane busy.  The order of evaluation is fixed, so sums stay
// deterministic.
#pragma once

#include "common.h"

constexpr int kPairQueue = 128;   // entries per wave: one full batch + one batch's overflow

// Neighbour-list entry: cell-order position in the low 30 bits, flags above.
constexpr unsigned kNbrSameGroup = 0x80000000u;   // partner in the atom's exclusion group
constexpr unsigned kNbrSite = 0x40000000u;        // partner's atom index is divisible by 3
constexpr unsigned kNbrIndex = 0x3fffffffu;

struct PairQueue {
  double dx[kPairQueue], dy[kPairQueue], dz[kPairQueue], r2[kPairQueue], q[kPairQueue];
};

__device__ __forceinline__ double min_img(double d, double box, double inv_box) { return d - box * rint(d * inv_box); }

// Orders this wave's LDS accesses: what a lane wrote before is visible to
// every lane of the wave after.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cell index of a coordinate triple (nc cells per edge).
__device__ __forceinline__ void cell_of(double x, double y, double z, double box, int nc, int* c) {
  const double xs[3] = {x, y, z};
  const double inv_box = 1.0 / box;
  for (int d = 0; d < 3; d++) {
    double s = xs[d] * inv_box;
    s -= floor(s);
    int ci = (int)(s * nc);
    c[d] = ci >= nc ? nc - 1 : ci;
  }
}

// Candidate range number `r` of the atom in cell c[] (wave-uniform):
// nc >= 3: the 9 x-rows of the 3x3 (y, z) neighbourhood, each one range
// (three cells contiguous in cell order) or, where the row wraps around the
// box, three ranges (pieces 0..2 of that row); nc < 3: the whole list.
// Returns false past the last range.
__device__ __forceinline__ bool candidate_range(int r, const int* c, int nc, const int* __restrict__ cstart,
                                                int* lo, int* hi) {
  if (nc < 3) {
    if (r > 0) return false;
    *lo = cstart[0];
    *hi = cstart[nc * nc * nc];
    return true;
  }
  const bool split = !(c[0] >= 1 && c[0] + 1 < nc);
  const int per_row = split ? 3 : 1;
  const int row = r / per_row, piece = r - row * per_row;
  if (row >= 9) return false;
  const int oz = row / 3 - 1, oy = row % 3 - 1;
  const int cy = (c[1] + oy + nc) % nc, cz = (c[2] + oz + nc) % nc;
  const int base = (cz * nc + cy) * nc;
  if (!split) {
    *lo = cstart[base + c[0] - 1];
    *hi = cstart[base + c[0] + 2];
  } else {
    const int cx = (c[0] + piece - 1 + nc) % nc;
    *lo = cstart[base + cx];
    *hi = cstart[base + cx + 1];
  }
  return true;
}

// Evaluates the first min(count, 64) queued pairs, one per lane, moves the
// rest to the front of the queue and returns how many remain.
template <class Pair>
__device__ __forceinline__ int queue_flush(PairQueue& Q, int count, int lane, Pair& pair) {
  const int nproc = count < 64 ? count : 64;
  wave_sync_lds();
  if (lane < nproc) pair(Q.dx[lane], Q.dy[lane], Q.dz[lane], Q.r2[lane], Q.q[lane]);
  const int rest = count - nproc;
  double v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0;
  if (lane < rest) {
    v0 = Q.dx[nproc + lane]; v1 = Q.dy[nproc + lane]; v2 = Q.dz[nproc + lane];
    v3 = Q.r2[nproc + lane]; v4 = Q.q[nproc + lane];
  }
  wave_sync_lds();
  if (lane < rest) {
    Q.dx[lane] = v0; Q.dy[lane] = v1; Q.dz[lane] = v2; Q.r2[lane] = v3; Q.q[lane] = v4;
  }
  wave_sync_lds();
  return rest;
}

// Pairs (i, j) of the atom at cell-order position wi, for every j within
// the neighbour cells with accept(jj, r2) true (jj = j's cell-order
// position; the caller maps it to an atom index when it needs one).
// pair(dx, dy, dz, r2, q_j) accumulates into the caller's per-lane sums.
// All lanes of the wave must call this together.  One loop with a single
// enqueue and a single evaluation site keeps the register count low.
template <class Accept, class Pair>
__device__ __forceinline__ void for_each_pair(int wi, double xi, double yi, double zi, double box, int nc,
                                              const int* __restrict__ cstart, const double4* __restrict__ spos,
                                              PairQueue& Q, Accept accept, Pair pair) {
  const int lane = threadIdx.x & 63;
  const double inv_box = 1.0 / box;
  int c[3];
  cell_of(xi, yi, zi, box, nc, c);
  int count = 0;          // wave-uniform queue length
  int r = 0, b0 = 0, hi = 0;
  bool more = candidate_range(0, c, nc, cstart, &b0, &hi);
  while (more && b0 >= hi) more = candidate_range(++r, c, nc, cstart, &b0, &hi);
  for (;;) {
    if (count >= 64 || (!more && count > 0)) {
      count = queue_flush(Q, count, lane, pair);
      continue;
    }
    if (!more) break;
    const int jj = b0 + lane;
    bool ok = false;
    double dx = 0, dy = 0, dz = 0, r2 = 0, qj = 0;
    if (jj < hi && jj != wi) {
      const double4 a = spos[jj];
      dx = min_img(xi - a.x, box, inv_box);
      dy = min_img(yi - a.y, box, inv_box);
      dz = min_img(zi - a.z, box, inv_box);
      r2 = dx * dx + dy * dy + dz * dz;
      qj = a.w;
      ok = accept(jj, r2);
    }
    const unsigned long long m = __ballot(ok);
    if (ok) {
      const int slot = count + __popcll(m & ((1ull << lane) - 1ull));
      Q.dx[slot] = dx; Q.dy[slot] = dy; Q.dz[slot] = dz; Q.r2[slot] = r2; Q.q[slot] = qj;
    }
    count += __popcll(m);
    b0 += 64;
    while (more && b0 >= hi) more = candidate_range(++r, c, nc, cstart, &b0, &hi);
  }
}

// The pairs of the cnt entries of one atom's neighbour list `ent`, for every
// entry with accept(entry, r2) true (accept sees the entry's flag bits).
// Most entries of a list lie within the cutoff, so each lane evaluates its
// own entries (k = lane, lane + 64, ...) in place, without the queue.
template <class Accept, class Pair>
__device__ __forceinline__ void for_each_listed(const int* __restrict__ ent, int cnt, double xi, double yi, double zi,
                                                double box, const double4* __restrict__ spos, Accept accept,
                                                Pair pair) {
  const double inv_box = 1.0 / box;
  for (int k = threadIdx.x & 63; k < cnt; k += 64) {
    const unsigned e = (unsigned)ent[k];
    const double4 a = spos[e & kNbrIndex];
    const double dx = min_img(xi - a.x, box, inv_box);
    const double dy = min_img(yi - a.y, box, inv_box);
    const double dz = min_img(zi - a.z, box, inv_box);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (accept(e, r2)) pair(dx, dy, dz, r2, a.w);
  }
}

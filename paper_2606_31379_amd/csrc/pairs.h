// Neighbour enumeration shared by the pair kernels (one wave per atom).
//
// Atoms are read from a cell-ordered packed copy {x, y, z, q} (built once per
// step after the cell sort), so the candidates of the three cells of one x
// row are one contiguous range (split only where the row wraps around the
// box) and are loaded coalesced, two batches of 64 in flight per lane.  Each
// lane applies the minimum image and the caller's acceptance test (cutoff,
// exclusions); accepted pairs are appended, in candidate order, to a per-wave
// queue in LDS (ballot + prefix rank), and the pair function -- the
// expensive part, e.g. erfc and exp in FP64 -- runs once per 64 queued pairs
// with every lane busy.  The order of evaluation is fixed, so sums stay
// deterministic.
#pragma once

#include "common.h"

constexpr int kPairQueue = 192;   // entries per wave: one full batch + two batches' overflow

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

// Pairs (i, j) of the atom at cell-order position wi, for every j within
// the neighbour cells with accept(jj, r2) true (jj = j's cell-order
// position; the caller maps it to an atom index when it needs one).
// pair(dx, dy, dz, r2, q_j) accumulates into the caller's per-lane sums.
// All lanes of the wave must call this together.
template <class Accept, class Pair>
__device__ __forceinline__ void for_each_pair(int wi, double xi, double yi, double zi, double box, int nc,
                                              const int* __restrict__ cstart, const double4* __restrict__ spos,
                                              PairQueue& Q, Accept accept, Pair pair) {
  const int lane = threadIdx.x & 63;
  const double inv_box = 1.0 / box;
  int c[3];
  cell_of(xi, yi, zi, box, nc, c);
  int count = 0;   // wave-uniform queue length
  auto drain = [&](int nproc) {
    // lanes < nproc evaluate entries 0..nproc-1, then the rest moves down
    wave_sync_lds();
    if (lane < nproc) pair(Q.dx[lane], Q.dy[lane], Q.dz[lane], Q.r2[lane], Q.q[lane]);
    const int rest = count - nproc;
    double v[2][5];
    for (int h = 0; h < 2; h++) {
      const int src = nproc + lane + 64 * h;
      if (lane + 64 * h < rest) {
        v[h][0] = Q.dx[src]; v[h][1] = Q.dy[src]; v[h][2] = Q.dz[src]; v[h][3] = Q.r2[src]; v[h][4] = Q.q[src];
      }
    }
    wave_sync_lds();
    for (int h = 0; h < 2; h++) {
      const int dst = lane + 64 * h;
      if (dst < rest) {
        Q.dx[dst] = v[h][0]; Q.dy[dst] = v[h][1]; Q.dz[dst] = v[h][2]; Q.r2[dst] = v[h][3]; Q.q[dst] = v[h][4];
      }
    }
    wave_sync_lds();
    count = rest;
  };
  // one batch of 64 candidates starting at b (< hi): test, enqueue
  auto push = [&](int b, int hi, const double4& a) {
    const int jj = b + lane;
    bool ok = false;
    double dx = 0, dy = 0, dz = 0, r2 = 0;
    if (jj < hi && jj != wi) {
      dx = min_img(xi - a.x, box, inv_box);
      dy = min_img(yi - a.y, box, inv_box);
      dz = min_img(zi - a.z, box, inv_box);
      r2 = dx * dx + dy * dy + dz * dz;
      ok = accept(jj, r2);
    }
    const unsigned long long m = __ballot(ok);
    if (ok) {
      const int slot = count + __popcll(m & ((1ull << lane) - 1ull));
      Q.dx[slot] = dx;
      Q.dy[slot] = dy;
      Q.dz[slot] = dz;
      Q.r2[slot] = r2;
      Q.q[slot] = a.w;
    }
    count += __popcll(m);
  };
  auto scan_range = [&](int lo, int hi) {
    for (int b0 = lo; b0 < hi; b0 += 128) {
      const int j0 = b0 + lane, j1 = b0 + 64 + lane;
      const double4 a0 = j0 < hi ? spos[j0] : make_double4(0, 0, 0, 0);
      const double4 a1 = j1 < hi ? spos[j1] : make_double4(0, 0, 0, 0);
      push(b0, hi, a0);
      if (b0 + 64 < hi) push(b0 + 64, hi, a1);
      if (count >= 64) drain(64);
      if (count >= 64) drain(64);
    }
  };
  if (nc < 3) {
    scan_range(cstart[0], cstart[nc * nc * nc]);
  } else {
    for (int oz = -1; oz <= 1; oz++)
      for (int oy = -1; oy <= 1; oy++) {
        const int cy = (c[1] + oy + nc) % nc, cz = (c[2] + oz + nc) % nc;
        const int row = (cz * nc + cy) * nc;
        if (c[0] >= 1 && c[0] + 1 < nc) {
          scan_range(cstart[row + c[0] - 1], cstart[row + c[0] + 2]);
        } else {
          for (int ox = -1; ox <= 1; ox++) {
            const int cx = (c[0] + ox + nc) % nc;
            scan_range(cstart[row + cx], cstart[row + cx + 1]);
          }
        }
      }
  }
  while (count > 0) drain(count < 64 ? count : 64);
}

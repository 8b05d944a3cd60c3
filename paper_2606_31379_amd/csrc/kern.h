// Kernel form shared by the single-system and the batched (many-replica)
// drivers.
//
// Every kernel is a struct K with
//   struct Args { ... };                      plain arguments of one system
//   static constexpr int kThreads;            workgroup size
//   __device__ static void run(const Args&, Grid);
// where Grid is the logical workgroup index and the number of workgroups the
// system's launch has.  k_one<K> launches it for one system (arguments by
// value); k_many<K> launches it for many independent systems at once: the
// systems' workgroups are laid end to end in one grid (no idle workgroups
// for the smaller systems), each workgroup finds its system by a binary
// search over the packed arguments in device memory.  The same run()
// therefore gives bitwise the same result for a system whether it runs alone
// or inside a batch.
//
// Launch sites call go<K>(args, grid, lds, stream).  Normally that launches
// k_one<K>.  While a Recorder is installed (batch set-up) it appends the
// packed arguments to the recorder instead, under the current sequence key,
// so the batch can merge the launch sequences of all its systems by key.
#pragma once
#include <type_traits>

#include <cstddef>
#include <cstring>
#include <vector>

#include "common.h"

struct Grid {
  int b;   // logical (XCD-renumbered) workgroup index
  int g;   // workgroups of this system's launch
};

// Contiguous chunk of [0, count) owned by workgroup G.b of G.g (reduction
// kernels on a capped grid); chunks are multiples of the block size.
__device__ __forceinline__ void chunk_range(const Grid& G, int64_t count, int* lo, int* hi) {
  int64_t per = (count + G.g - 1) / G.g;
  per = (per + kRedBlock - 1) / kRedBlock * kRedBlock;
  const int64_t l = (int64_t)G.b * per;
  *lo = (int)(l < count ? l : count);
  *hi = (int)(l + per < count ? l + per : count);
}

template <class K>
struct Packed {
  typename K::Args a;
  int grid;   // workgroups of this system's launch
  int off;    // first workgroup of this system in the batched grid
};

// Occupancy floor of a kernel family: K::kWavesPerEu waves per SIMD when
// it names one (the register budget follows), else none.
template <class K, class = void>
struct WavesPerEu {
  static constexpr int v = 1;
};
template <class K>
struct WavesPerEu<K, std::void_t<decltype(K::kWavesPerEu)>> {
  static constexpr int v = K::kWavesPerEu;
};

template <class K>
__global__ void __launch_bounds__(K::kThreads, WavesPerEu<K>::v) k_one(typename K::Args a) {
  K::run(a, Grid{xcd_block(), (int)gridDim.x});
}

// The XCD renumbering runs over the whole batched grid, so each system's
// workgroups stay on few XCDs, in logical order.
template <class K>
__global__ void __launch_bounds__(K::kThreads, WavesPerEu<K>::v) k_many(const Packed<K>* __restrict__ p, int count) {
  const int lam = xcd_block();
  int lo = 0, hi = count - 1;   // last system whose first workgroup is <= lam (uniform)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (p[mid].off <= lam) lo = mid;
    else hi = mid - 1;
  }
  const int b = lam - p[lo].off, g = p[lo].grid;
  if (b >= g) return;   // padding of the grid to a multiple of 8
  const typename K::Args a = p[lo].a;   // uniform: scalar loads
  K::run(a, Grid{b, g});
}

// Launches k_many<K> over `count` packed argument sets at `dev` with `gx`
// workgroups in all.
using ManyFn = hipError_t (*)(const void* dev, int count, int gx, size_t lds, hipStream_t s);
template <class K>
hipError_t launch_many(const void* dev, int count, int gx, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_many<K>, dim3(gx), dim3(K::kThreads), lds, s, (const Packed<K>*)dev, count);
  return hipGetLastError();
}

// One recorded launch of one system.
struct LaunchRec {
  uint32_t key;                     // merge key (sequence position class)
  ManyFn many;                      // batched launcher of the kernel
  int grid;                         // workgroups of this system's launch
  size_t lds;                       // dynamic LDS bytes
  size_t off_field;                 // byte offset of Packed<K>::off
  std::vector<unsigned char> args;  // Packed<K> bytes
};

struct Recorder {
  uint32_t base = 0, seq = 0;
  std::vector<LaunchRec> recs;
};

// The recorder of the batch being set up on this host thread (null: launch).
extern thread_local Recorder* g_recorder;

// Start a new key class: launches that follow get keys base*64 + 0, 1, ...
inline void rec_key(uint32_t base) {
  if (g_recorder) {
    g_recorder->base = base;
    g_recorder->seq = 0;
  }
}

template <class K>
hipError_t go(const typename K::Args& a, int grid, size_t lds, hipStream_t s) {
  if (g_recorder) {
    Packed<K> p{a, grid, 0};
    LaunchRec r;
    r.key = g_recorder->base * 64u + g_recorder->seq++;
    r.many = &launch_many<K>;
    r.grid = grid;
    r.lds = lds;
    r.off_field = offsetof(Packed<K>, off);
    r.args.resize(sizeof p);
    memcpy(r.args.data(), &p, sizeof p);
    g_recorder->recs.push_back(std::move(r));
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_one<K>, dim3(grid), dim3(K::kThreads), lds, s, a);
  return hipGetLastError();
}

// Raise the dynamic-LDS limit of both launch forms of K to at least `bytes`.
template <class K>
hipError_t allow_lds(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_one<K>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_many<K>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

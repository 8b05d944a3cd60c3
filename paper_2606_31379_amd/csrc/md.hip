// Molecular-dynamics support kernels: velocity-Verlet kicks and drift, the
// non-electrostatic terms of the two model systems, and the energy log.
#include <algorithm>

#include "kern.h"
#include "launch.h"
#include "pairs.h"

namespace {

constexpr int kBlock = 256;

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64-bit multiplies
// on the 128-bit counter, the 64-bit key bumped by the Weyl constants
// between rounds.
__device__ __forceinline__ void philox4x32_10(unsigned x[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    const unsigned long long p0 = 0xD2511F53ull * x[0], p1 = 0xCD9E8D57ull * x[2];
    const unsigned y0 = (unsigned)(p1 >> 32) ^ x[1] ^ k0, y1 = (unsigned)p1;
    const unsigned y2 = (unsigned)(p0 >> 32) ^ x[3] ^ k1, y3 = (unsigned)p0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Standard normal number d (0..2) of atom a at thermostat step `step`, end
// `half` of the step: counter {a, step low, step high, half}, key = seed;
// uniforms (x + 1/2) 2^-32, then the Box-Muller transform of the pairs
// (u0, u1) -> normals 0, 1 and (u2, u3) -> normal 2.
__device__ __forceinline__ double thermo_normal(const Thermostat& T, int a, long long step, int half, int d) {
  unsigned x[4] = {(unsigned)a, (unsigned)(unsigned long long)step, (unsigned)((unsigned long long)step >> 32),
                   (unsigned)half};
  philox4x32_10(x, T.seed0, T.seed1);
  const double s = 1.0 / 4294967296.0;
  const unsigned ur = d < 2 ? x[0] : x[2], ua = d < 2 ? x[1] : x[3];
  const double r = sqrt(-2.0 * log(((double)ur + 0.5) * s));
  const double ang = 2.0 * M_PI * (((double)ua + 0.5) * s);
  return d == 1 ? r * sin(ang) : r * cos(ang);
}

// One thread per velocity component.  drift: the start of a step (the
// thermostat's first half, the half kick, the drift); otherwise its end
// (the half kick, the thermostat's second half).
struct KickDrift {
  struct Args {
    int n_atoms, drift;
    double dt, f2a;
    double *pos, *vel;
    const double *f, *mass;
    Thermostat th;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void KickDrift::run(const Args& A, Grid G) {
  const int n_atoms = A.n_atoms, drift = A.drift;
  const double dt = A.dt, f2a = A.f2a;
  double* __restrict__ pos = A.pos;
  double* __restrict__ vel = A.vel;
  const double* __restrict__ f = A.f;
  const double* __restrict__ mass = A.mass;
  const int t = G.b * kBlock + threadIdx.x;
  if (t >= 3 * n_atoms) return;
  const int a = t / 3;
  const Thermostat& T = A.th;
  double v = vel[t];
  if (drift && T.on)
    v = T.a * v + T.b * sqrt(T.kt / (mass[a] * T.mv2e)) * thermo_normal(T, a, T.ctl->therm_step, 0, t - 3 * a);
  v += 0.5 * dt * f[t] / mass[a] * f2a;
  if (!drift && T.on)
    v = T.a * v + T.b * sqrt(T.kt / (mass[a] * T.mv2e)) * thermo_normal(T, a, T.ctl->therm_step, 1, t - 3 * a);
  vel[t] = v;
  if (drift) pos[t] += dt * v;
}

__device__ __forceinline__ double mi(double d, double box, double inv_box) { return d - box * rint(d * inv_box); }

// model 1: stand-in Born-Mayer repulsion between all pairs (shifted at r_cut);
// model 2: flexible three-site water -- intermolecular O-O Lennard-Jones
// (shifted at r_cut) plus harmonic O-H bonds and H-O-H angle.
//
// Pair terms: each wave takes `span` (1..64) consecutive cell-order
// positions, finds the atoms with pair terms among them (all atoms in model
// 1, the O atoms in model 2) by ballot, and runs them one after another:
// lanes stride the atom's neighbour list (or its neighbour cells), a fixed
// shuffle tree sums the lanes.  force += F_pair.  Large systems take 64
// positions per wave, so no wave is spent on an H atom; small ones fewer,
// so there are still enough waves to fill the chip.
struct NonElec {
  struct Args {
    int n_atoms, model, nc, span;
    double box, rc2, p0, p1;
    const int *cstart, *cperm;
    const double4* spos;   // cell-ordered {x, y, z, q}
    double *force, *partial;
    const int *list, *nlist;   // neighbour lists as in the short-range kernel (null: scan the cells)
    int cap;
    int skip_listed;           // 1: atoms with a list are done by the short-range list pass
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void NonElec::run(const Args& A, Grid G) {
  const int n_atoms = A.n_atoms, model = A.model, nc = A.nc;
  const double box = A.box, rc2 = A.rc2, p0 = A.p0, p1 = A.p1;
  const int* __restrict__ cstart = A.cstart;
  const int* __restrict__ cperm = A.cperm;
  double* __restrict__ force = A.force;
  __shared__ double sh[kBlock / 64];
  __shared__ PairQueue queue[kBlock / 64];
  const int lane = threadIdx.x & 63;
  const int nwaves = G.g * (kBlock / 64);
  PairQueue& Q = queue[threadIdx.x >> 6];
  double en = 0.0;
  double shift;
  if (model == 1) {
    shift = p0 * exp(-sqrt(rc2) / p1);
  } else {
    const double s2 = p1 * p1 / rc2, s6 = s2 * s2 * s2;
    shift = 4.0 * p0 * (s6 * s6 - s6);
  }
  const int span = A.span;
  for (int chunk = (G.b * kBlock + threadIdx.x) >> 6; chunk * span < n_atoms && model != 0; chunk += nwaves) {
    const int mine = chunk * span + lane;
    const bool in = lane < span && mine < n_atoms;
    const int ai = in ? cperm[mine] : 0;
    const bool listed = A.skip_listed && in && A.list && A.nlist[mine] <= A.cap;
    unsigned long long todo = __ballot(in && !listed && (model == 1 || ai % 3 == 0));
    while (todo) {
      const int l = __ffsll((unsigned long long)todo) - 1;   // wave-uniform
      todo &= todo - 1;
      const int wave = chunk * span + l;
      const int i = __shfl(ai, l, 64);
      const double4 me = A.spos[wave];
      const double xi = me.x, yi = me.y, zi = me.z;
      double fx = 0.0, fy = 0.0, fz = 0.0;
      auto pair = [&](double dx, double dy, double dz, double r2, double) {
        double f;
        if (model == 1) {
          const double r = sqrt(r2);
          const double v = p0 * exp(-r / p1);
          f = v / p1 / r;
          en += 0.5 * (v - shift);
        } else {
          const double sr2 = p1 * p1 / r2;
          const double sr6 = sr2 * sr2 * sr2;
          f = 24.0 * p0 * (2.0 * sr6 * sr6 - sr6) / r2;
          en += 0.5 * (4.0 * p0 * (sr6 * sr6 - sr6) - shift);
        }
        fx += f * dx; fy += f * dy; fz += f * dz;
      };
      const int nl = A.list ? A.nlist[wave] : 0;
      if (A.list && nl <= A.cap)
        // model 2: the list's site flag marks O atoms; the O of the atom's
        // own molecule is the atom itself, which no list holds
        for_each_listed(A.list + (size_t)wave * A.cap, nl, xi, yi, zi, box, A.spos,
                        [&](unsigned e, double r2) { return r2 < rc2 && (model == 1 || (e & kNbrSite)); }, pair);
      else
        for_each_pair(
            wave, xi, yi, zi, box, nc, cstart, A.spos, Q,
            [&](int jj, double r2) {
              if (!(r2 < rc2)) return false;
              if (model == 1) return true;
              const int j = cperm[jj];
              return j % 3 == 0 && j / 3 != i / 3;
            },
            pair);
      fx = wave_sum(fx);
      fy = wave_sum(fy);
      fz = wave_sum(fz);
      if (lane == 0) {
        force[3 * i] += fx;
        force[3 * i + 1] += fy;
        force[3 * i + 2] += fz;
      }
    }
  }
  en = wave_sum(en);
  if (lane == 0) sh[threadIdx.x >> 6] = en;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kBlock / 64; k++) s += sh[k];
    A.partial[G.b] = s;
  }
}

// Bonded terms of model 2, one thread per atom: the harmonic O-H bonds and
// H-O-H angle of the atom's molecule that act on it (each atom recomputes
// its molecule's geometry; no atomics); the molecule's energy is counted at
// its O.  force += F_bonded.
struct Bonded {
  struct Args {
    int n_atoms;
    double box, k_bond, r0, k_angle, theta0;
    const double* pos;
    double *force, *partial;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void Bonded::run(const Args& A, Grid G) {
  const double box = A.box, inv_box = 1.0 / box, p2 = A.k_bond, p3 = A.r0, p4 = A.k_angle, p5 = A.theta0;
  const double* __restrict__ pos = A.pos;
  __shared__ double sh[kBlock / 64];
  double en = 0.0;
  for (int i = G.b * kBlock + threadIdx.x; i < A.n_atoms; i += G.g * kBlock) {
    const int o = (i / 3) * 3;
    double a[3], b[3];
    for (int d = 0; d < 3; d++) {
      a[d] = mi(pos[3 * (o + 1) + d] - pos[3 * o + d], box, inv_box);
      b[d] = mi(pos[3 * (o + 2) + d] - pos[3 * o + d], box, inv_box);
    }
    const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double fa = -p2 * (la - p3) / la, fb = -p2 * (lb - p3) / lb;
    double cth = (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / (la * lb);
    cth = fmin(1.0, fmax(-1.0, cth));
    const double th = acos(cth);
    const double sth = fmax(sqrt(1.0 - cth * cth), 1e-12);
    const double g = p4 * (th - p5) / sth;
    double f1[3], f2[3];
    for (int d = 0; d < 3; d++) {
      f1[d] = fa * a[d] + g * (b[d] / (la * lb) - cth * a[d] / (la * la));
      f2[d] = fb * b[d] + g * (a[d] / (la * lb) - cth * b[d] / (lb * lb));
    }
    const int role = i - o;
    double fx, fy, fz;
    if (role == 0) {
      fx = -(f1[0] + f2[0]); fy = -(f1[1] + f2[1]); fz = -(f1[2] + f2[2]);
      en += 0.5 * p2 * ((la - p3) * (la - p3) + (lb - p3) * (lb - p3)) + 0.5 * p4 * (th - p5) * (th - p5);
    } else {
      const double* fr = role == 1 ? f1 : f2;
      fx = fr[0]; fy = fr[1]; fz = fr[2];
    }
    A.force[3 * i] += fx;
    A.force[3 * i + 1] += fy;
    A.force[3 * i + 2] += fz;
  }
  const double bs = block_sum(en, sh);
  if (threadIdx.x == 0) A.partial[G.b] = bs;
}

struct FinOther {
  struct Args {
    int nb;
    const double* partial;
    double* e_out;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid) {
    __shared__ double sh[kBlock / 64];
    const double tot = reduce_partials_sum(A.partial, A.nb, sh);
    if (threadIdx.x == 0) *A.e_out = tot;
  }
};

struct Kinetic {
  struct Args {
    int n_atoms;
    double mv2e;
    const double *vel, *mass;
    double* partial;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G) {
    __shared__ double sh[kBlock / 64];
    const double* __restrict__ vel = A.vel;
    const double* __restrict__ mass = A.mass;
    double ke = 0.0;
    for (int a = G.b * kBlock + threadIdx.x; a < A.n_atoms; a += G.g * kBlock) {
      const double vx = vel[3 * a], vy = vel[3 * a + 1], vz = vel[3 * a + 2];
      ke += 0.5 * mass[a] * (vx * vx + vy * vy + vz * vz) * A.mv2e;
    }
    const double bs = block_sum(ke, sh);
    if (threadIdx.x == 0) A.partial[G.b] = bs;
  }
};

// Log row ctl->md_step of the energy/cycle logs, then advance the row.
struct FinLog {
  struct Args {
    int nb;
    const double *partial, *e4, *e_other;
    double* log_base;
    int* clog_base;
    Ctl* ctl;
  };
  static constexpr int kThreads = kBlock;
  __device__ static void run(const Args& A, Grid G);
};
__device__ void FinLog::run(const Args& A, Grid) {
  const double* __restrict__ e4 = A.e4;
  const double* __restrict__ e_other = A.e_other;
  double* log_base = A.log_base;
  int* clog_base = A.clog_base;
  Ctl* ctl = A.ctl;
  __shared__ double sh[kBlock / 64];
  const double tot = reduce_partials_sum(A.partial, A.nb, sh);
  if (threadIdx.x == 0) {
    const int k = ctl->md_step;
    if (log_base) {
      double* row = log_base + 6 * (size_t)k;
      row[0] = e4[0]; row[1] = e4[1]; row[2] = e4[2]; row[3] = *e_other; row[4] = tot;
      row[5] = e4[3] + *e_other + tot;
    }
    if (clog_base) clog_base[k] = ctl->cycles;
    ctl->md_step = k + 1;
    ctl->therm_step++;
  }
}

}  // namespace

hipError_t launch_kick_drift(int n_atoms, double* pos, double* vel, const double* force, const double* mass,
                             double dt, double f2a, int drift, hipStream_t s, const Thermostat* th) {
  const Thermostat off{0, 1.0, 0.0, 0.0, 1.0, 0u, 0u, nullptr};
  return go<KickDrift>({n_atoms, drift, dt, f2a, pos, vel, force, mass, th ? *th : off},
                       blocks_for(3 * (int64_t)n_atoms, kBlock), 0, s);
}

hipError_t launch_nonelec(int n_atoms, const double* pos, double box, double r_cut, int model, double p0,
                          double p1, double p2, double p3, double p4, double p5, int nc, const int* cstart,
                          const int* cperm, const void* spos, double* force, double* partial, double* e_out,
                          hipStream_t s, const int* list, const int* nlist, int cap, int prior, int skip_listed) {
  // positions per wave: 64, halved while that leaves fewer than 8192 waves
  int span = 64;
  while (span > 1 && (n_atoms + span - 1) / span < 8192) span >>= 1;
  const int64_t waves = (n_atoms + span - 1) / span;
  // partials: `prior` of the short-range list pass, the pair kernel's, then the bonded kernel's
  const int nb = std::min(blocks_for(waves * 64, kBlock), kPartialSlots - kMaxRedBlocks);
  hipError_t e = go<NonElec>({n_atoms, model, nc, span, box, r_cut * r_cut, p0, p1, cstart, cperm,
                              (const double4*)spos, force, partial + prior, list, nlist, cap, skip_listed}, nb, 0, s);
  if (e != hipSuccess) return e;
  int nbb = 0;
  if (model == 2) {
    nbb = std::min(blocks_for(n_atoms, kBlock), kMaxRedBlocks);
    e = go<Bonded>({n_atoms, box, p2, p3, p4, p5, pos, force, partial + prior + nb}, nbb, 0, s);
    if (e != hipSuccess) return e;
  }
  return go<FinOther>({prior + nb + nbb, partial, e_out}, 1, 0, s);
}

hipError_t launch_kinetic_log(int n_atoms, const double* vel, const double* mass, double mv2e,
                              const double* energy4, const double* e_other, double* log_base, int* clog_base,
                              Ctl* ctl, double* partial, hipStream_t s) {
  const int nb = std::min(blocks_for(n_atoms, kBlock), kMaxRedBlocks);
  hipError_t e = go<Kinetic>({n_atoms, mv2e, vel, mass, partial}, nb, 0, s);
  if (e != hipSuccess) return e;
  return go<FinLog>({nb, partial, energy4, e_other, log_base, clog_base, ctl}, 1, 0, s);
}

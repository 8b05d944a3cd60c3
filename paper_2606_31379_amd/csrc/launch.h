// Host-side launchers of the kernels, one function per kernel family.
// Every launcher enqueues on `s` and returns the launch status.
#pragma once

#include "common.h"

// Kernel families that can be timed individually with HIP events.
enum KernelId {
  KT_HALFSWEEP = 0, KT_OUTER = 1, KT_SMOOTH = 2, KT_RESTRICT = 3, KT_PROLONG = 4, KT_SWEEP0 = 5,
  KT_TAIL = 6, KT_SPREAD = 7, KT_GATHER = 8, KT_SR = 9, KT_SIGMA = 10, KT_PHI = 11, KT_FUSED_DOWN = 12,
  KT_FUSED_UP = 13, KT_COUNT = 14
};
// Bracket one launch of kernel family `id` on multigrid level `level` with
// events when that family/level is being timed (no-ops otherwise).
// `bytes` is the launch's algorithmic HBM traffic.
void kt_begin(int id, int level, hipStream_t s);
void kt_end(int id, int level, double bytes, hipStream_t s);

// ---- particles (particles.hip) ------------------------------------------
// Tile key of each atom (the tile holding its first stencil index); slot =
// arrival rank inside the key's bin.
hipError_t launch_bin_tiles(int n_atoms, const double* pos, double box, int n, int p, int tile, int ntx, int* key,
                           int* slot, int* count, Ctl* ctl, hipStream_t s);
// Cell key of each atom for the short-range cell list (nc cells per edge).
// gate (here and in the scan, scatter, sort and pack below): non-null makes
// the launch do nothing unless *gate (the neighbour-list rebuild flag).
hipError_t launch_bin_cells(int n_atoms, const double* pos, double box, int nc, int* key, int* slot,
                            int* count, Ctl* ctl, hipStream_t s, const int* gate = nullptr);
// Exclusive scan of count[0..nbins) into start[0..nbins], zeroing count;
// bsum needs scan_partials(nbins) ints.
int scan_partials(int nbins);
hipError_t launch_scan(int nbins, int* count, int* start, int* bsum, hipStream_t s, const int* gate = nullptr);
// perm_raw[start[key[a]] + slot[a]] = a.
hipError_t launch_scatter(int n_atoms, const int* key, const int* slot, const int* start, int* perm_raw,
                          hipStream_t s, const int* gate = nullptr);
// Sort every bin's atom list by atom index (makes all later sums deterministic).
hipError_t launch_sort_bins(int nbins, const int* start, const int* perm_raw, int* perm, Ctl* ctl,
                            hipStream_t s, const int* gate = nullptr);
// Sort every bin's atom list by (class, atom index) and write each atom's
// records at its sorted position i: rb[i] = {stencil origin x | y << 10 |
// z << 20, atom index} (int2), rq[i] = {charge, tau_x, tau_y, tau_z}
// (double4); cls[8 b + c] = first position of class c (the faces of its tile
// the atom's stencil crosses: bit d for axis d) in bin b.
hipError_t launch_sort_pack(int nbins, const int* start, const int* perm_raw, int n_atoms, const double* pos,
                            const double* qa, double box, int n, int p, int tile, void* rb, void* rq, int* cls,
                            hipStream_t s);
// Owner-computes spread: q (natural layout, FP64 or FP32) from the binned atoms.
hipError_t launch_spread(bool fp64, int n, int p, int tile, int ntx, double box, const int* start, const int* cls,
                         const void* rb, const void* rq, void* q, hipStream_t s);
// Long-range force and energy by interpolating the central-difference
// gradient of phi (precision of phi: fp64 or float): two-point, or
// four-point with stencil 1 (orders p <= 5).
// phi: FP64 mode reads the new potential from phi0/phi1 (selected on the
// device), mixed mode reads the FP32 copy phi32.
// finalize = false launches the per-atom kernel only (back-to-back timing);
// with finalize, both kernels do nothing unless ctl->done (the step's solve
// has converged), so they may be enqueued before the host has checked it.
hipError_t launch_gather(bool fp64, int n_atoms, int n, int p, int tile, int ntx, double h, double k_e,
                         const int* start, const void* rb, const void* rq, const double* phi0, const double* phi1,
                         const float* phi32, double* force, double* partial, Ctl* ctl, hipStream_t s,
                         bool finalize = true, int stencil = 0);
// Short-range erfc pairs (neighbour lists or the cell list), exclusion correction, energy
// assembly into energy_out[4] (may be NULL).  force += F_sr; the sum of the
// final forces goes to ctl->net_force (nfpart: 3 * kPartialSlots doubles).
// spos[jj] = {x, y, z, q} of atom cperm[jj] (cell order), for the pair kernels.
hipError_t launch_cell_pack(int n_atoms, const int* cperm, const double* pos, const double* qa, void* spos,
                            hipStream_t s, const int* gate = nullptr);
// Neighbour lists with a skin.  Check (every step): spos[jj] = the atom
// cperm[jj] now (the order of the last build), and ctl->nbr_stale = 1 when
// some atom has moved more than skin/2 from ref[jj] (double4).  Build (does
// nothing unless ctl->nbr_stale): on a cell list of cells at least r_list
// wide, list[wi * cap ..] = entries (cell-order index | flag bits) of every
// atom within r_list of atom wi, nlist[wi] = their number (may exceed cap:
// then the pair kernels scan the cells for wi), ref = spos.
hipError_t launch_nbr_check(int n_atoms, double box, double skin, const int* cperm, const double* pos,
                            const double* qa, void* spos, const void* ref, Ctl* ctl, hipStream_t s);
hipError_t launch_nbr_build(int n_atoms, double box, double r_list, int nc, int excl_group, int cap,
                            const int* cstart, const int* cperm, const void* spos, void* ref, int* list, int* nlist,
                            Ctl* ctl, hipStream_t s);
// erfc_tab: erfcx table for alpha r in [0, alpha r_cut] (erfc_n intervals,
// erfc_scale intervals per unit).  list/nlist/cap: neighbour lists as built
// by launch_nbr_build (null: every atom scans the cells).  ne_model != 0
// (lists only): the list pass also adds the MD pair term (1: Born-Mayer
// A = ne_p0, rho = ne_p1; 2: O-O Lennard-Jones eps, sigma) to force, its
// energy partials in nepart[0 .. *ne_written); atoms over capacity are left
// to launch_nonelec.
hipError_t launch_sr(int n_atoms, const double* pos, const double* qa, double box, double alpha,
                     double r_cut, double k_e, int nc, int excl_group, const int* cstart,
                     const int* cperm, const void* spos, const double* erfc_tab, int erfc_n, double erfc_scale,
                     double* force, double e_self, double* energy_out, double* partial, double* nfpart, Ctl* ctl,
                     hipStream_t s, const int* list = nullptr, const int* nlist = nullptr, int cap = 0,
                     int ne_model = 0, double ne_p0 = 0.0, double ne_p1 = 0.0, double* nepart = nullptr,
                     int* ne_written = nullptr);

// ---- mesh (mesh.hip) -----------------------------------------------------
// Folded periodic smoothing filter along one axis: out = sum_m c[m] v[i+m-K],
// launch shape `tile` (see smooth_tile_shape; 0 = default); taps, in and
// out in FP64 or FP32.
hipError_t launch_smooth(bool fp64, int n, int axis, int tile, int ntaps, int half, const void* taps,
                         const void* in, void* out, hipStream_t s);
int smooth_tile_count();
bool smooth_tile_ok(int tile, int n, int ntaps);
void smooth_tile_shape(int tile, int* lines_per_workgroup, int* outputs_per_thread);
// stencil 1 (fourth order): sigma_p = (h/4pi) A phi_p + B q^s and the outer
// residual with the 19-point A (see the kernels).
// sigma_p = (h/4pi) M (2 phi^k - phi^{k-1}) + q^s (cold: q^s) and the
// multiplier predictor into y; a one-workgroup pass then forms the mean of
// sigma_p, max|q^s| and the threshold and opens the solve.  History buffers
// are selected on the device from the control block.
// qs: the smoothed charges in FP32 (qs32) or FP64.
hipError_t launch_sigma(int n, double h, bool qs32, const void* qs, const double* phi0, const double* phi1,
                        const double* yb0, const double* yb1, const double* yb2, double* sigma, double* y,
                        double tol, int tol_mode, double* partial, Ctl* ctl, hipStream_t s, bool finalize = true,
                        int stencil = 0);
// Outer FP64 residual r = sigma - mean - M y: cycle 0 (first) on the
// predicted y in y0; cycle c > 0 on y + e, the previous cycle's y (y0 or y1
// by parity) plus this cycle's correction, written to the other buffer; r
// written colour-split in T for the next V-cycle; it marks its stop decision
// pending, and with finalize a one-workgroup pass makes it right away
// (res_hist[c], done/status and which buffer holds y).
// spart (first residual only): sigma's partials, reduced by every workgroup
// in place of the separate FinSigma pass (tol, tol_mode: the threshold).
hipError_t launch_outer(bool fp64, int n, int first, int max_cycles, const double* sigma, double* y0, double* y1,
                        const void* e0, const void* e1, void* r0, void* r1, double* partial, Ctl* ctl,
                        hipStream_t s, bool finalize = true, const double* spart = nullptr, double tol = 0.0,
                        int tol_mode = 0, int stencil = 0);
// The stop decision of an outer residual: its partials (nb workgroups,
// max then sum) on a fine mesh of n3 points, with the cycle cap.
struct Decide {
  const double* partial;
  int nb, n3, max_cycles;
};
struct LevelBufs {
  int n;
  void* e0; void* e1;   // colour-split correction
  void* r0; void* r1;   // colour-split right-hand side
  // fused legs (fty > 0): tiles of fty x ftz rows; the down leg writes d0/d1,
  // the up leg reads d1 and writes e0/e1
  void* d0 = nullptr; void* d1 = nullptr;
  int fty = 0, ftz = 0;
  // the two post-smoothing sweeps as one walk (post_sweeps_fused) write the
  // level's final correction here instead of e0/e1
  void* s0 = nullptr; void* s1 = nullptr;
};
// True when the V-cycle's post-smoothing on level buffers b runs as one
// walk (FP32 512^3 or 256^3 finest levels of single systems, two sweeps after the black-only
// prolongation): the level's correction after the cycle is then in s0/s1.
bool post_sweeps_fused(const LevelBufs& b, bool fp64, int nu2);
// The colour-split buffers holding the finest level's correction after a V-cycle.
inline const void* cycle_e0(const LevelBufs& b, bool fp64, int nu2) {
  return post_sweeps_fused(b, fp64, nu2) ? b.s0 : b.e0;
}
inline const void* cycle_e1(const LevelBufs& b, bool fp64, int nu2) {
  return post_sweeps_fused(b, fp64, nu2) ? b.s1 : b.e1;
}
// Largest level edge that gets the fused-leg buffers.
constexpr int kFusedEdgeMax = 64;
// Tile rows of a fused level of edge n (0: the level is not fused).
int fused_tile(int n);
// One V-cycle on the colour-split level hierarchy lv[0..levels-1]; the
// levels from `tail` on run in one LDS-resident workgroup; levels with
// fty > 0 run each leg as one fused launch when its LDS box fits.  With
// `decide`, the tail first makes the pending stop decision of the previous
// outer residual (the launches before it may run on a system that has just
// converged: they only write scratch levels).
hipError_t launch_vcycle(bool fp64, const LevelBufs* lv, int levels, int tail, int nu1, int nu2,
                         const double* green, Ctl* ctl, hipStream_t s, const Decide* decide = nullptr);
// One finest-level launch of a V-cycle kernel family (KT_HALFSWEEP, KT_SWEEP0,
// KT_RESTRICT, KT_PROLONG, KT_TAIL) on the current buffers; *bytes = its
// algorithmic traffic.
hipError_t launch_vcycle_kernel(bool fp64, int kid, const LevelBufs* lv, int levels, int tail, int nu1, int nu2,
                                const double* green, Ctl* ctl, hipStream_t s, double* bytes);
// phi update and history push: phi^{k+1} = phi_p - (4pi/h)(y - mean y);
// buffers selected on the device.  With `decide`, every workgroup first makes
// the pending stop decision of the last outer residual (the first records it).
hipError_t launch_phi_update(int n, double h, double* phi0, double* phi1, const double* ya, const double* yb,
                             double* yh0, double* yh1, double* yh2, float* phi32, Ctl* ctl, hipStream_t s,
                             const Decide* decide = nullptr);
// Persistent launch of `phases` finest-level half-sweeps (colours
// alternating) on every system of a batch, with per-system device barriers
// between them (a measurement of that form against one batched launch per
// sweep).  d_sys: device buffer for the per-system arguments (*sys_bytes
// reports the size; uploaded when `upload`); d_work: 2 + n_sys * phases ints
// (work[1] becomes 1 if a wait gave up).  grid: resident workgroups.
hipError_t persist_halfsweeps(bool fp64, const LevelBufs* const* lv0, Ctl* const* ctls, int n_sys, int phases,
                              void* d_sys, int* d_work, int grid, hipStream_t s, size_t* sys_bytes, bool upload);
int persist_grid();
size_t persist_sys_bytes(bool fp64, int n_sys);
// End-of-step rotation of the history on the device.
hipError_t launch_advance(Ctl* ctl, hipStream_t s);
// Layout conversions for inspection and the stand-alone V-cycle.
hipError_t launch_widen(bool fp64, int64_t count, const void* in, double* out, hipStream_t s);
hipError_t launch_cs_to_nat(bool fp64, int n, const void* c0, const void* c1, double* out, hipStream_t s);
hipError_t launch_nat_to_cs(bool fp64, int n, const double* in, void* c0, void* c1, hipStream_t s);
hipError_t launch_set_ctl_open(Ctl* ctl, hipStream_t s);
// out = in - *sub (device scalar).
hipError_t launch_sub_scalar(int64_t count, const double* in, double* out, const double* sub, hipStream_t s);
hipError_t tail_configure(bool fp64, int n_tail, int levels_tail, size_t* lds_bytes);
// Allows the smoothing kernels the LDS they need on an n^3 mesh.
hipError_t smooth_configure();
// Allows the fused-leg kernels and the shared-row column walk (sigma_p,
// outer residual) their LDS.
hipError_t fused_configure();

// ---- molecular dynamics (md.hip) ----------------------------------------
// th (null: none): the OVRVO thermostat halves at the two ends of the step.
hipError_t launch_kick_drift(int n_atoms, double* pos, double* vel, const double* force,
                             const double* mass, double dt, double f2a, int drift, hipStream_t s,
                             const Thermostat* th = nullptr);
hipError_t launch_nonelec(int n_atoms, const double* pos, double box, double r_cut, int model,
                          double p0, double p1, double p2, double p3, double p4, double p5,
                          int nc, const int* cstart, const int* cperm, const void* spos, double* force,
                          double* partial, double* e_out, hipStream_t s, const int* list = nullptr,
                          const int* nlist = nullptr, int cap = 0, int prior = 0, int skip_listed = 0);
// Kinetic energy and one row (ctl->md_step, then advanced) of the logs.
hipError_t launch_kinetic_log(int n_atoms, const double* vel, const double* mass, double mv2e,
                              const double* energy4, const double* e_other, double* log_base,
                              int* clog_base, Ctl* ctl, double* partial, hipStream_t s);

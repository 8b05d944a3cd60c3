// Host side of the library: planning, workspace allocation, the per-step
// launch sequence and the C ABI declared in include/p3maze.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "launch.h"
#include "p3maze.h"

namespace {

thread_local std::string g_last_error;

p3mz_status fail(p3mz_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

p3mz_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_last_error = buf;
  return e == hipErrorOutOfMemory ? P3MZ_ERR_OUT_OF_MEMORY : P3MZ_ERR_HIP;
}

constexpr double kPi = 3.14159265358979323846;
constexpr int kTile = 8;

struct Plan {
  int n = 0, p = 0, levels = 0, tail = 0, K = 0;
  double h = 0, sigma = 0, sigma_s2 = 0, nu_s = 0;
};

// Derived parameters of the method: spacing, Gaussian width (alpha =
// 1/(sqrt(2) sigma)), smoothing variance sigma^2 - p h^2/6 split into K
// diffusion steps of weight nu <= 1/4, and the multigrid levels N/2^l down
// to 4^3.
p3mz_status make_plan(const p3mz_params& P, Plan* pl) {
  if (!(P.box > 0) || !(P.alpha > 0) || !(P.r_cut > 0) || P.r_cut > 0.5 * P.box)
    return fail(P3MZ_ERR_INVALID_ARG, "box, alpha and r_cut must be positive with r_cut <= box/2");
  if (P.order < 2 || P.order > P3MZ_MAX_ORDER) return fail(P3MZ_ERR_INVALID_ARG, "order must be in 2..7");
  if (!(P.tol > 0) || P.tol_mode < 0 || P.tol_mode > 1) return fail(P3MZ_ERR_INVALID_ARG, "bad tolerance");
  if (P.max_cycles < 0 || P.max_cycles > P3MZ_MAX_CYCLES) return fail(P3MZ_ERR_INVALID_ARG, "max_cycles must be in 0..64");
  if (P.predictor < 0 || P.predictor > 3) return fail(P3MZ_ERR_INVALID_ARG, "predictor must be in 0..3");
  if (P.precision != P3MZ_PREC_FP64 && P.precision != P3MZ_PREC_MIXED) return fail(P3MZ_ERR_INVALID_ARG, "bad precision");
  if (P.nu_pre < -1 || P.nu_post < -1 || P.nu_pre > 16 || P.nu_post > 16) return fail(P3MZ_ERR_INVALID_ARG, "bad sweep counts");
  if (P.excl_group < 0) return fail(P3MZ_ERR_INVALID_ARG, "excl_group must be >= 0");
  const int n = P.mesh;
  int m = n;
  while (m > 4 && (m & 1) == 0) m >>= 1;
  if (n < 8 || m != 4 || n > 512) return fail(P3MZ_ERR_MESH_SHAPE, "mesh must be 4*2^m points per edge, 8..512");
  pl->n = n;
  pl->p = P.order;
  pl->h = P.box / n;
  pl->sigma = 1.0 / (sqrt(2.0) * P.alpha);
  pl->sigma_s2 = pl->sigma * pl->sigma - P.order * pl->h * pl->h / 6.0;
  if (!(pl->sigma_s2 > 0)) return fail(P3MZ_ERR_MESH_SHAPE, "mesh spacing too coarse for the Gaussian width");
  pl->K = std::max(1, (int)ceil(2.0 * pl->sigma_s2 / (pl->h * pl->h)));
  pl->nu_s = pl->sigma_s2 / (2.0 * pl->K * pl->h * pl->h);
  pl->levels = 0;
  for (int q = n; q >= 4; q >>= 1) pl->levels++;
  pl->tail = 0;
  while ((n >> pl->tail) > P3MZ_TAIL_MAX) pl->tail++;
  return P3MZ_OK;
}

// Folded periodic taps of the K-fold convolution of [nu, 1-2nu, nu]:
// out[i] = sum_m taps[m] v[(i + m - half) mod n].
void smoothing_taps(int n, int K, double nu, std::vector<double>* taps, int* half) {
  std::vector<double> c(1, 1.0);
  for (int s = 0; s < K; s++) {
    std::vector<double> d(c.size() + 2, 0.0);
    for (size_t j = 0; j < c.size(); j++) {
      d[j] += nu * c[j];
      d[j + 1] += (1.0 - 2.0 * nu) * c[j];
      d[j + 2] += nu * c[j];
    }
    c.swap(d);
  }
  const int len = 2 * K + 1;
  if (len <= n) {
    *taps = c;
    *half = K;
  } else {
    taps->assign(n, 0.0);
    for (int j = 0; j < len; j++) {
      int off = ((j - K) % n + n) % n;
      (*taps)[off] += c[j];
    }
    *half = 0;
  }
}

// Periodic Green's function of M on the 4^3 mesh with the constant mode
// removed: G(x) = (1/64) sum_{k != 0} cos(2 pi k.x / 4) / lambda(k),
// lambda(k) = -4 sum_d sin^2(pi k_d / 4).
void coarse_green(double* g) {
  for (int z = 0; z < 4; z++)
    for (int y = 0; y < 4; y++)
      for (int x = 0; x < 4; x++) {
        double s = 0.0;
        for (int c = 0; c < 4; c++)
          for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
              if (a == 0 && b == 0 && c == 0) continue;
              const double sa = sin(kPi * a / 4), sb = sin(kPi * b / 4), sc = sin(kPi * c / 4);
              const double lam = -4.0 * (sa * sa + sb * sb + sc * sc);
              s += cos(2.0 * kPi * (a * x + b * y + c * z) / 4.0) / lam;
            }
        g[(z * 4 + y) * 4 + x] = s / 64.0;
      }
}

}  // namespace

struct p3mz_ctx {
  p3mz_params P{};
  Plan pl;
  int dev = 0;
  bool fp64 = true;
  size_t tsz = 8;
  int nu1 = 2, nu2 = 2;
  int64_t n_atoms = 0;
  int64_t n3 = 0;
  double e_self = 0;
  int ntaps = 0, half = 0;
  // device buffers
  void* d_taps = nullptr;
  double* d_green = nullptr;
  double* d_qa = nullptr;
  int *d_base = nullptr, *d_key = nullptr, *d_slot = nullptr, *d_perm_raw = nullptr, *d_perm = nullptr;
  void* d_w = nullptr;
  int ntx = 0, nbins = 0;
  int *d_count = nullptr, *d_start = nullptr;
  int nc = 1, ncells = 1;
  int *d_ckey = nullptr, *d_cslot = nullptr, *d_ccount = nullptr, *d_cstart = nullptr, *d_cperm_raw = nullptr,
      *d_cperm = nullptr;
  void *d_q = nullptr, *d_qs = nullptr, *d_tmp = nullptr;
  double* d_sigma = nullptr;
  double* d_y[2] = {nullptr, nullptr};
  double* d_phi[2] = {nullptr, nullptr};
  double* d_yh[3] = {nullptr, nullptr, nullptr};
  float* d_phi32 = nullptr;
  LevelBufs lv[P3MZ_MAX_LEVELS];
  double* d_partial = nullptr;
  Ctl* d_ctl = nullptr;
  Ctl* h_ctl = nullptr;
  double* d_energy = nullptr;   // internal energy4 when the caller passes none
  double* d_vscratch = nullptr; // FP64 natural buffer for p3mz_vcycle
  // md
  double* d_md_force = nullptr;
  double* d_e_other = nullptr;
  bool md_have_force = false;
  // history
  int have_hist = 0, n_yh = 0, k_idx = 0;
  int yh_order[3] = {0, 1, 2};   // newest first
  int last_cycles = 0;
  int64_t steps = 0;
  p3mz_stats st{};
  std::vector<void*> allocs;
  // optional timing: stage events and one kernel family's per-launch events
  bool timing = false;
  hipEvent_t stage_ev[5] = {};
  int kt_id = -1;
  std::vector<hipEvent_t> kt_ev;
  std::vector<double> kt_bytes;
  int kt_used = 0;
  double kt_total_ms = 0.0, kt_total_bytes = 0.0;
  int64_t kt_launches = 0;

  template <typename T>
  p3mz_status alloc(T** p, size_t count) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc", __FILE__, __LINE__);
    allocs.push_back(v);
    *p = (T*)v;
    return P3MZ_OK;
  }
  p3mz_status allocb(void** p, size_t bytes) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(bytes, 1));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc", __FILE__, __LINE__);
    allocs.push_back(v);
    *p = v;
    return P3MZ_OK;
  }
  ~p3mz_ctx() {
    for (void* v : allocs) (void)hipFree(v);
    if (h_ctl) (void)hipHostFree(h_ctl);
    for (hipEvent_t e : stage_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : kt_ev) (void)hipEventDestroy(e);
  }
};

// The context whose compute is being enqueued (kernel-timer hooks read it).
static p3mz_ctx* g_active = nullptr;

void kt_begin(int id, int level, hipStream_t s) {
  p3mz_ctx* c = g_active;
  if (!c || c->kt_id != id || level != 0 || c->kt_used + 2 > (int)c->kt_ev.size()) return;
  (void)hipEventRecord(c->kt_ev[c->kt_used], s);
}

void kt_end(int id, int level, double bytes, hipStream_t s) {
  p3mz_ctx* c = g_active;
  if (!c || c->kt_id != id || level != 0 || c->kt_used + 2 > (int)c->kt_ev.size()) return;
  (void)hipEventRecord(c->kt_ev[c->kt_used + 1], s);
  c->kt_bytes[c->kt_used / 2] = bytes;
  c->kt_used += 2;
}

namespace {

#define P3MZ_TRY(expr)              \
  do {                              \
    p3mz_status s_ = (expr);        \
    if (s_ != P3MZ_OK) return s_;   \
  } while (0)

p3mz_status setup(p3mz_ctx* c, const double* charges_host) {
  const Plan& pl = c->pl;
  const int n = pl.n;
  c->n3 = (int64_t)n * n * n;
  c->fp64 = c->P.precision == P3MZ_PREC_FP64;
  c->tsz = c->fp64 ? 8 : 4;
  c->nu1 = c->P.nu_pre >= 0 ? c->P.nu_pre : 2;
  c->nu2 = c->P.nu_post >= 0 ? c->P.nu_post : 2;
  if (c->nu1 + c->nu2 < 1) return fail(P3MZ_ERR_INVALID_ARG, "nu_pre + nu_post must be >= 1");
  P3MZ_HIP_TRY(hipGetDevice(&c->dev));
  // charges
  double e_self = 0.0;
  for (int64_t a = 0; a < c->n_atoms; a++) e_self -= c->P.coulomb_k * c->P.alpha / sqrt(kPi) * charges_host[a] * charges_host[a];
  c->e_self = e_self;
  P3MZ_TRY(c->alloc(&c->d_qa, c->n_atoms));
  P3MZ_HIP_TRY(hipMemcpy(c->d_qa, charges_host, sizeof(double) * c->n_atoms, hipMemcpyHostToDevice));
  // smoothing taps
  std::vector<double> taps;
  smoothing_taps(n, pl.K, pl.nu_s, &taps, &c->half);
  c->ntaps = (int)taps.size();
  // The charge source (weights, spread, smoothing, sigma_p) is FP64 in both
  // modes: FP32 rounding of q^s (~1e-7 relative) would exceed the residual
  // tolerance and change the V-cycle counts of the warm-started solve.
  P3MZ_TRY(c->allocb(&c->d_taps, taps.size() * 8));
  P3MZ_HIP_TRY(hipMemcpy(c->d_taps, taps.data(), taps.size() * 8, hipMemcpyHostToDevice));
  double g[64];
  coarse_green(g);
  P3MZ_TRY(c->alloc(&c->d_green, 64));
  P3MZ_HIP_TRY(hipMemcpy(c->d_green, g, sizeof g, hipMemcpyHostToDevice));
  // atoms / bins
  const int64_t na = c->n_atoms;
  c->ntx = n / kTile;
  c->nbins = c->ntx * c->ntx * c->ntx;
  P3MZ_TRY(c->alloc(&c->d_base, 3 * na));
  P3MZ_TRY(c->allocb(&c->d_w, (size_t)3 * na * pl.p * 8));
  P3MZ_TRY(c->alloc(&c->d_key, na));
  P3MZ_TRY(c->alloc(&c->d_slot, na));
  P3MZ_TRY(c->alloc(&c->d_perm_raw, na));
  P3MZ_TRY(c->alloc(&c->d_perm, na));
  P3MZ_TRY(c->alloc(&c->d_count, c->nbins));
  P3MZ_TRY(c->alloc(&c->d_start, c->nbins + 1));
  P3MZ_HIP_TRY(hipMemset(c->d_count, 0, sizeof(int) * c->nbins));
  c->nc = (int)floor(c->P.box / c->P.r_cut);
  if (c->nc < 3) c->nc = 1;
  if (c->nc > 256) c->nc = 256;
  c->ncells = c->nc * c->nc * c->nc;
  P3MZ_TRY(c->alloc(&c->d_ckey, na));
  P3MZ_TRY(c->alloc(&c->d_cslot, na));
  P3MZ_TRY(c->alloc(&c->d_cperm_raw, na));
  P3MZ_TRY(c->alloc(&c->d_cperm, na));
  P3MZ_TRY(c->alloc(&c->d_ccount, c->ncells));
  P3MZ_TRY(c->alloc(&c->d_cstart, c->ncells + 1));
  P3MZ_HIP_TRY(hipMemset(c->d_ccount, 0, sizeof(int) * c->ncells));
  // mesh
  const size_t n3 = (size_t)c->n3;
  P3MZ_TRY(c->allocb(&c->d_q, n3 * 8));
  P3MZ_TRY(c->allocb(&c->d_qs, n3 * 8));
  P3MZ_TRY(c->allocb(&c->d_tmp, n3 * 8));
  P3MZ_TRY(c->alloc(&c->d_sigma, n3));
  for (int i = 0; i < 2; i++) P3MZ_TRY(c->alloc(&c->d_y[i], n3));
  for (int i = 0; i < 2; i++) {
    P3MZ_TRY(c->alloc(&c->d_phi[i], n3));
    P3MZ_HIP_TRY(hipMemset(c->d_phi[i], 0, n3 * 8));
  }
  for (int i = 0; i < 3; i++) P3MZ_TRY(c->alloc(&c->d_yh[i], n3));
  if (!c->fp64) P3MZ_TRY(c->alloc(&c->d_phi32, n3));
  for (int l = 0; l < pl.levels; l++) {
    const int nl = n >> l;
    const size_t half = (size_t)nl * nl * nl / 2;
    LevelBufs& b = c->lv[l];
    b.n = nl;
    P3MZ_TRY(c->allocb(&b.e0, half * c->tsz));
    P3MZ_TRY(c->allocb(&b.e1, half * c->tsz));
    P3MZ_TRY(c->allocb(&b.r0, half * c->tsz));
    P3MZ_TRY(c->allocb(&b.r1, half * c->tsz));
  }
  const size_t max_blocks = (std::max<size_t>(n3, (size_t)na) + 255) / 256 + 1;
  P3MZ_TRY(c->alloc(&c->d_partial, 2 * max_blocks));
  P3MZ_TRY(c->alloc(&c->d_ctl, 1));
  P3MZ_HIP_TRY(hipMemset(c->d_ctl, 0, sizeof(Ctl)));
  P3MZ_HIP_TRY(hipHostMalloc((void**)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  memset(c->h_ctl, 0, sizeof(Ctl));
  P3MZ_TRY(c->alloc(&c->d_energy, 4));
  P3MZ_TRY(c->alloc(&c->d_md_force, 3 * na));
  P3MZ_TRY(c->alloc(&c->d_e_other, 1));
  size_t lds = 0;
  P3MZ_HIP_TRY(tail_configure(c->fp64, n >> pl.tail, pl.levels - pl.tail, &lds));
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  return P3MZ_OK;
}

p3mz_status finish_step(p3mz_ctx* c, hipStream_t s) {
  P3MZ_HIP_TRY(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  P3MZ_HIP_TRY(hipStreamSynchronize(s));
  return P3MZ_OK;
}

// The step: bin + sort atoms, spread, smooth, constraint at the prediction,
// V-cycles until the FP64 residual meets the tolerance, field update,
// gather, short-range pairs.
p3mz_status compute_step(p3mz_ctx* c, const double* pos, double* force, double* energy, hipStream_t s) {
  const Plan& pl = c->pl;
  const int n = pl.n, na = (int)c->n_atoms;
  const bool f64 = c->fp64;
  const double N3 = (double)c->n3, ts = (double)c->tsz;
  g_active = c;
  struct Reset { ~Reset() { g_active = nullptr; } } reset_active;
  auto stage = [&](int i) {
    if (c->timing) (void)hipEventRecord(c->stage_ev[i], s);
  };
  stage(0);
  // 1. binning and deterministic order
  P3MZ_HIP_TRY(launch_bin_stencil(true, na, pos, c->P.box, n, pl.p, kTile, c->ntx, c->d_base, c->d_w, c->d_key,
                                  c->d_slot, c->d_count, c->d_ctl, s));
  P3MZ_HIP_TRY(launch_scan(c->nbins, c->d_count, c->d_start, s));
  P3MZ_HIP_TRY(launch_scatter(na, c->d_key, c->d_slot, c->d_start, c->d_perm_raw, s));
  P3MZ_HIP_TRY(launch_sort_bins(c->nbins, c->d_start, c->d_perm_raw, c->d_perm, c->d_ctl, s));
  // 2. spread and smoothing
  kt_begin(KT_SPREAD, 0, s);
  P3MZ_HIP_TRY(launch_spread(true, n, pl.p, kTile, c->ntx, c->d_start, c->d_perm, c->d_base, c->d_w, c->d_qa, c->d_q, s));
  kt_end(KT_SPREAD, 0, 8.0 * N3 + (double)na * (24.0 * pl.p + 24.0), s);
  kt_begin(KT_SMOOTH, 0, s);
  P3MZ_HIP_TRY(launch_smooth(true, n, 0, c->ntaps, c->half, c->d_taps, c->d_q, c->d_qs, s));
  kt_end(KT_SMOOTH, 0, 16.0 * N3, s);
  kt_begin(KT_SMOOTH, 0, s);
  P3MZ_HIP_TRY(launch_smooth(true, n, 1, c->ntaps, c->half, c->d_taps, c->d_qs, c->d_tmp, s));
  kt_end(KT_SMOOTH, 0, 16.0 * N3, s);
  kt_begin(KT_SMOOTH, 0, s);
  P3MZ_HIP_TRY(launch_smooth(true, n, 2, c->ntaps, c->half, c->d_taps, c->d_tmp, c->d_qs, s));
  kt_end(KT_SMOOTH, 0, 16.0 * N3, s);
  stage(1);
  // 3. constraint at the Verlet prediction and multiplier predictor
  const int cold = !c->have_hist;
  const int m_eff = cold ? 0 : std::min(c->P.predictor, c->n_yh);
  double* pk = c->d_phi[c->k_idx];
  double* pkm1 = c->d_phi[1 - c->k_idx];
  kt_begin(KT_SIGMA, 0, s);
  P3MZ_HIP_TRY(launch_sigma(true, n, pl.h, cold, m_eff, c->d_qs, pk, pkm1, c->d_yh[c->yh_order[0]],
                            c->d_yh[c->yh_order[1]], c->d_yh[c->yh_order[2]], c->d_sigma, c->d_y[0], c->P.tol,
                            c->P.tol_mode, c->d_partial, c->d_ctl, s));
  kt_end(KT_SIGMA, 0, (cold ? 24.0 : 40.0 + 8.0 * m_eff) * N3, s);
  // 4. V-cycles; the host enqueues the expected number of cycles, then
  // checks the device flag and continues one cycle at a time if needed.
  const LevelBufs& f = c->lv[0];
  kt_begin(KT_OUTER, 0, s);
  P3MZ_HIP_TRY(launch_outer(f64, n, 0, c->P.max_cycles, c->d_sigma, c->d_y[0], c->d_y[0], f.e0, f.e1, f.r0, f.r1,
                            c->d_partial, c->d_ctl, s));
  kt_end(KT_OUTER, 0, (16.0 + ts) * N3, s);
  int cyc = 1;
  int batch = std::max(1, c->last_cycles);
  while (cyc <= c->P.max_cycles) {
    for (int b = 0; b < batch && cyc <= c->P.max_cycles; b++, cyc++) {
      P3MZ_HIP_TRY(launch_vcycle(f64, c->lv, pl.levels, pl.tail, c->nu1, c->nu2, c->d_green, c->d_ctl, s));
      kt_begin(KT_OUTER, 0, s);
      P3MZ_HIP_TRY(launch_outer(f64, n, cyc, c->P.max_cycles, c->d_sigma, c->d_y[(cyc - 1) & 1], c->d_y[cyc & 1],
                                f.e0, f.e1, f.r0, f.r1, c->d_partial, c->d_ctl, s));
      kt_end(KT_OUTER, 0, (24.0 + 2.0 * ts) * N3, s);
    }
    if (cyc > c->P.max_cycles) break;
    P3MZ_HIP_TRY(hipMemcpyAsync(&c->h_ctl->done, &c->d_ctl->done, sizeof(int), hipMemcpyDeviceToHost, s));
    P3MZ_HIP_TRY(hipStreamSynchronize(s));
    if (c->h_ctl->done) break;
    batch = 1;
  }
  // 5. field update and history
  kt_begin(KT_PHI, 0, s);
  if (cold) {
    P3MZ_HIP_TRY(launch_phi_update(n, pl.h, 1, pk, pkm1, c->d_y[0], c->d_y[1], pk, pkm1, nullptr, c->d_phi32,
                                   c->d_ctl, s));
  } else {
    const int slot = c->yh_order[2];
    P3MZ_HIP_TRY(launch_phi_update(n, pl.h, 0, pk, pkm1, c->d_y[0], c->d_y[1], pkm1, nullptr, c->d_yh[slot],
                                   c->d_phi32, c->d_ctl, s));
  }
  kt_end(KT_PHI, 0, (cold ? 16.0 : 40.0) * N3 + (f64 ? 0.0 : 4.0 * N3), s);
  stage(2);
  // 6. gather on the new potential, short-range pairs, energies
  const double* phi_new = cold ? pk : pkm1;
  const void* phi_read = f64 ? (const void*)phi_new : (const void*)c->d_phi32;
  kt_begin(KT_GATHER, 0, s);
  P3MZ_HIP_TRY(launch_gather(f64, na, n, pl.p, pl.h, c->P.coulomb_k, c->d_perm, c->d_base, c->d_w, c->d_qa, phi_read,
                             force, c->d_partial, c->d_ctl, s));
  const double pe = pl.p + 2.0;
  kt_end(KT_GATHER, 0, (double)na * (48.0 + 24.0 * pl.p + pe * pe * pe * (f64 ? 8.0 : 4.0)), s);
  stage(3);
  P3MZ_HIP_TRY(launch_bin_cells(na, pos, c->P.box, c->nc, c->d_ckey, c->d_cslot, c->d_ccount, c->d_ctl, s));
  P3MZ_HIP_TRY(launch_scan(c->ncells, c->d_ccount, c->d_cstart, s));
  P3MZ_HIP_TRY(launch_scatter(na, c->d_ckey, c->d_cslot, c->d_cstart, c->d_cperm_raw, s));
  P3MZ_HIP_TRY(launch_sort_bins(c->ncells, c->d_cstart, c->d_cperm_raw, c->d_cperm, c->d_ctl, s));
  kt_begin(KT_SR, 0, s);
  P3MZ_HIP_TRY(launch_sr(na, pos, c->d_qa, c->P.box, c->P.alpha, c->P.r_cut, c->P.coulomb_k, c->nc, c->P.excl_group,
                         c->d_cstart, c->d_cperm, force, c->e_self, energy ? energy : c->d_energy,
                         c->d_partial, c->d_ctl, s));
  kt_end(KT_SR, 0, (double)na * 56.0, s);
  stage(4);
  P3MZ_TRY(finish_step(c, s));
  if (c->timing) {
    float ms[4];
    for (int i = 0; i < 4; i++) P3MZ_HIP_TRY(hipEventElapsedTime(&ms[i], c->stage_ev[i], c->stage_ev[i + 1]));
    for (int i = 0; i < 4; i++) c->st.ms_stage[i] = ms[i];
  }
  for (int i = 0; i + 1 < c->kt_used; i += 2) {
    float ms = 0.f;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->kt_ev[i], c->kt_ev[i + 1]));
    c->kt_total_ms += ms;
    c->kt_total_bytes += c->kt_bytes[i / 2];
    c->kt_launches++;
  }
  c->kt_used = 0;
  const Ctl& h = *c->h_ctl;
  if (h.nan_flag) {
    P3MZ_HIP_TRY(hipMemsetAsync(&c->d_ctl->nan_flag, 0, sizeof(int), s));
    c->have_hist = 0;
    c->n_yh = 0;
    return fail(P3MZ_ERR_NAN, "non-finite position");
  }
  // history bookkeeping (mirrors the device writes above)
  if (cold) {
    c->n_yh = 0;
  } else {
    c->k_idx = 1 - c->k_idx;
    const int slot = c->yh_order[2];
    c->yh_order[2] = c->yh_order[1];
    c->yh_order[1] = c->yh_order[0];
    c->yh_order[0] = slot;
    c->n_yh = std::min(3, c->n_yh + 1);
  }
  c->have_hist = 1;
  c->last_cycles = h.cycles;
  c->steps++;
  p3mz_stats& st = c->st;
  st.status = h.status ? P3MZ_WARN_NOT_CONVERGED : P3MZ_OK;
  st.cycles = h.cycles;
  st.cold = cold;
  st.m_eff = m_eff;
  st.nu_pre = c->nu1;
  st.nu_post = c->nu2;
  st.K = pl.K;
  st.levels = pl.levels;
  st.nu_smooth = pl.nu_s;
  st.thresh = h.thresh;
  st.norm_qs = h.norm_qs;
  for (int i = 0; i <= P3MZ_MAX_CYCLES; i++) st.res_hist[i] = i <= h.cycles ? h.res_hist[i] : 0.0;
  st.e_sr = h.e_sr;
  st.e_lr = h.e_lr;
  st.e_self = c->e_self;
  st.e_total = h.e_sr + h.e_lr + c->e_self;
  st.steps = c->steps;
  if (h.status) {
    g_last_error = "V-cycle cap reached before the tolerance";
    return P3MZ_WARN_NOT_CONVERGED;
  }
  return P3MZ_OK;
}

}  // namespace

extern "C" {

p3mz_status p3mz_create(const p3mz_params* params, int64_t n_atoms, const double* charges_host, p3mz_ctx** out) {
  if (!out) return fail(P3MZ_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!params || !charges_host || n_atoms < 1 || n_atoms > (1LL << 30))
    return fail(P3MZ_ERR_INVALID_ARG, "params/charges NULL or n_atoms out of range");
  Plan pl;
  P3MZ_TRY(make_plan(*params, &pl));
  double sq = 0.0, sa = 0.0;
  for (int64_t a = 0; a < n_atoms; a++) {
    if (!isfinite(charges_host[a])) return fail(P3MZ_ERR_INVALID_ARG, "non-finite charge");
    sq += charges_host[a];
    sa += fabs(charges_host[a]);
  }
  if (fabs(sq) > 1e-10 * sa) return fail(P3MZ_ERR_NOT_NEUTRAL, "total charge is not zero");
  p3mz_ctx* c = new (std::nothrow) p3mz_ctx();
  if (!c) return fail(P3MZ_ERR_OUT_OF_MEMORY, "context allocation");
  c->P = *params;
  c->pl = pl;
  c->n_atoms = n_atoms;
  p3mz_status s = setup(c, charges_host);
  if (s != P3MZ_OK) {
    delete c;
    return s;
  }
  *out = c;
  return P3MZ_OK;
}

p3mz_status p3mz_compute(p3mz_ctx* ctx, const double* pos_dev, double* force_dev, double* energy_dev, void* stream) {
  if (!ctx || !pos_dev) return fail(P3MZ_ERR_INVALID_ARG, "ctx or pos_dev is NULL");
  return compute_step(ctx, pos_dev, force_dev, energy_dev, (hipStream_t)stream);
}

p3mz_status p3mz_get_mesh(p3mz_ctx* ctx, int32_t which, double* out_dev, void* stream) {
  if (!ctx || !out_dev) return fail(P3MZ_ERR_INVALID_ARG, "ctx or out_dev is NULL");
  hipStream_t s = (hipStream_t)stream;
  const size_t n3 = (size_t)ctx->n3;
  switch (which) {
    case 0: P3MZ_HIP_TRY(launch_widen(true, n3, ctx->d_q, out_dev, s)); break;
    case 1: P3MZ_HIP_TRY(launch_widen(true, n3, ctx->d_qs, out_dev, s)); break;
    case 2: {
      // zero-mean sigma_p = stored sigma - mean (mean kept in the control block)
      P3MZ_HIP_TRY(launch_sub_scalar(n3, ctx->d_sigma, out_dev, &ctx->d_ctl->mean_sigma, s));
      break;
    }
    case 3: {
      // the final multiplier after the zero-mean projection is the newest history slot
      // on warm steps; on cold steps it is not stored, so it is rebuilt from phi.
      if (ctx->st.cold) return fail(P3MZ_ERR_STATE, "multiplier of a cold solve is not kept");
      P3MZ_HIP_TRY(hipMemcpyAsync(out_dev, ctx->d_yh[ctx->yh_order[0]], n3 * 8, hipMemcpyDeviceToDevice, s));
      break;
    }
    case 4: P3MZ_HIP_TRY(hipMemcpyAsync(out_dev, ctx->d_phi[ctx->k_idx], n3 * 8, hipMemcpyDeviceToDevice, s)); break;
    case 5: P3MZ_HIP_TRY(hipMemcpyAsync(out_dev, ctx->d_phi[1 - ctx->k_idx], n3 * 8, hipMemcpyDeviceToDevice, s)); break;
    default: return fail(P3MZ_ERR_INVALID_ARG, "unknown mesh id");
  }
  return P3MZ_OK;
}

p3mz_status p3mz_vcycle(p3mz_ctx* ctx, const double* r_dev, double* e_dev, void* stream) {
  if (!ctx || !r_dev || !e_dev) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const LevelBufs& f = ctx->lv[0];
  P3MZ_HIP_TRY(launch_set_ctl_open(ctx->d_ctl, s));
  P3MZ_HIP_TRY(launch_nat_to_cs(ctx->fp64, ctx->pl.n, r_dev, f.r0, f.r1, s));
  P3MZ_HIP_TRY(launch_vcycle(ctx->fp64, ctx->lv, ctx->pl.levels, ctx->pl.tail, ctx->nu1, ctx->nu2, ctx->d_green,
                             ctx->d_ctl, s));
  P3MZ_HIP_TRY(launch_cs_to_nat(ctx->fp64, ctx->pl.n, f.e0, f.e1, e_dev, s));
  return P3MZ_OK;
}

p3mz_status p3mz_get_stats(const p3mz_ctx* ctx, p3mz_stats* out) {
  if (!ctx || !out) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  *out = ctx->st;
  return P3MZ_OK;
}

p3mz_status p3mz_reset_history(p3mz_ctx* ctx) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  ctx->have_hist = 0;
  ctx->n_yh = 0;
  ctx->last_cycles = 0;
  ctx->md_have_force = false;
  return P3MZ_OK;
}

// blob: magic, n, precision, have_hist, n_yh, steps, last_cycles, then
// phi^k, phi^{k-1}, y^k, y^{k-1}, y^{k-2} (FP64, natural layout).
static const int64_t kMagic = 0x50334d5a53543031LL;   // "P3MZST01"

p3mz_status p3mz_save_state(const p3mz_ctx* ctx, void* host_buf, size_t* bytes) {
  if (!ctx || !bytes) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  const size_t n3 = (size_t)ctx->n3;
  const size_t need = 7 * sizeof(int64_t) + 5 * n3 * sizeof(double);
  if (!host_buf) {
    *bytes = need;
    return P3MZ_OK;
  }
  if (*bytes < need) return fail(P3MZ_ERR_INVALID_ARG, "buffer too small");
  int64_t hdr[7] = {kMagic, ctx->pl.n, ctx->P.precision, ctx->have_hist, ctx->n_yh, ctx->steps, ctx->last_cycles};
  char* b = (char*)host_buf;
  memcpy(b, hdr, sizeof hdr);
  b += sizeof hdr;
  const double* arr[5] = {ctx->d_phi[ctx->k_idx], ctx->d_phi[1 - ctx->k_idx], ctx->d_yh[ctx->yh_order[0]],
                          ctx->d_yh[ctx->yh_order[1]], ctx->d_yh[ctx->yh_order[2]]};
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  for (int i = 0; i < 5; i++) {
    P3MZ_HIP_TRY(hipMemcpy(b, arr[i], n3 * 8, hipMemcpyDeviceToHost));
    b += n3 * 8;
  }
  *bytes = need;
  return P3MZ_OK;
}

p3mz_status p3mz_load_state(p3mz_ctx* ctx, const void* host_buf, size_t bytes) {
  if (!ctx || !host_buf) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  const size_t n3 = (size_t)ctx->n3;
  const size_t need = 7 * sizeof(int64_t) + 5 * n3 * sizeof(double);
  if (bytes != need) return fail(P3MZ_ERR_STATE, "state blob has the wrong size");
  int64_t hdr[7];
  const char* b = (const char*)host_buf;
  memcpy(hdr, b, sizeof hdr);
  b += sizeof hdr;
  if (hdr[0] != kMagic || hdr[1] != ctx->pl.n || hdr[2] != ctx->P.precision || hdr[4] < 0 || hdr[4] > 3)
    return fail(P3MZ_ERR_STATE, "state blob does not match this context");
  ctx->k_idx = 0;
  ctx->yh_order[0] = 0;
  ctx->yh_order[1] = 1;
  ctx->yh_order[2] = 2;
  double* arr[5] = {ctx->d_phi[0], ctx->d_phi[1], ctx->d_yh[0], ctx->d_yh[1], ctx->d_yh[2]};
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  for (int i = 0; i < 5; i++) {
    P3MZ_HIP_TRY(hipMemcpy(arr[i], b, n3 * 8, hipMemcpyHostToDevice));
    b += n3 * 8;
  }
  ctx->have_hist = (int)hdr[3];
  ctx->n_yh = (int)hdr[4];
  ctx->steps = hdr[5];
  ctx->last_cycles = (int)hdr[6];
  ctx->md_have_force = false;
  return P3MZ_OK;
}

p3mz_status p3mz_md_run(p3mz_ctx* ctx, double* pos_dev, double* vel_dev, const double* mass_dev,
                        const p3mz_mdterms* terms, double dt, int32_t n_steps, double* energy_log_dev,
                        int32_t* cycles_log_dev, void* stream) {
  if (!ctx || !pos_dev || !vel_dev || !mass_dev || !terms || n_steps < 0 || !(dt > 0))
    return fail(P3MZ_ERR_INVALID_ARG, "bad md_run arguments");
  if (terms->model < 0 || terms->model > 2) return fail(P3MZ_ERR_INVALID_ARG, "unknown model");
  if (terms->model == 2 && ctx->n_atoms % 3 != 0)
    return fail(P3MZ_ERR_INVALID_ARG, "the water model needs O,H,H triples");
  hipStream_t s = (hipStream_t)stream;
  const int na = (int)ctx->n_atoms;
  double p[6] = {0, 0, 0, 0, 0, 0};
  if (terms->model == 1) {
    p[0] = terms->bm_a;
    p[1] = terms->bm_rho;
  } else if (terms->model == 2) {
    p[0] = terms->lj_eps; p[1] = terms->lj_sigma; p[2] = terms->k_bond; p[3] = terms->r0;
    p[4] = terms->k_angle; p[5] = terms->theta0;
  }
  auto forces = [&](double* e4) -> p3mz_status {
    p3mz_status st = compute_step(ctx, pos_dev, ctx->d_md_force, e4, s);
    if (st < 0) return st;
    // the cell list of the short-range pass is still valid for these positions
    hipError_t e = launch_nonelec(na, pos_dev, ctx->P.box, ctx->P.r_cut, terms->model, p[0], p[1], p[2], p[3], p[4],
                                  p[5], ctx->nc, ctx->d_cstart, ctx->d_cperm, ctx->d_md_force, ctx->d_partial,
                                  ctx->d_e_other, s);
    if (e != hipSuccess) return hip_fail(e, "launch_nonelec", __FILE__, __LINE__);
    return st;
  };
  p3mz_status worst = P3MZ_OK;
  if (!ctx->md_have_force) {
    p3mz_status st = forces(ctx->d_energy);
    if (st < 0) return st;
    ctx->md_have_force = true;
  }
  for (int step = 0; step < n_steps; step++) {
    P3MZ_HIP_TRY(launch_kick_drift(na, pos_dev, vel_dev, ctx->d_md_force, mass_dev, dt, terms->force_to_acc, 1, s));
    p3mz_status st = forces(ctx->d_energy);
    if (st < 0) return st;
    if (st > worst) worst = st;
    P3MZ_HIP_TRY(launch_kick_drift(na, pos_dev, vel_dev, ctx->d_md_force, mass_dev, dt, terms->force_to_acc, 0, s));
    P3MZ_HIP_TRY(launch_kinetic_log(na, vel_dev, mass_dev, terms->mv2_to_energy, ctx->d_energy, ctx->d_e_other,
                                    energy_log_dev ? energy_log_dev + 6 * (size_t)step : nullptr,
                                    cycles_log_dev ? cycles_log_dev + step : nullptr, ctx->d_ctl, ctx->d_partial, s));
  }
  P3MZ_HIP_TRY(hipStreamSynchronize(s));
  return worst;
}

p3mz_status p3mz_set_timing(p3mz_ctx* ctx, int32_t on) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (on && !ctx->stage_ev[0])
    for (hipEvent_t& e : ctx->stage_ev) P3MZ_HIP_TRY(hipEventCreate(&e));
  ctx->timing = on != 0;
  for (double& v : ctx->st.ms_stage) v = 0.0;
  return P3MZ_OK;
}

p3mz_status p3mz_set_kernel_timer(p3mz_ctx* ctx, int32_t kernel_id) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (kernel_id < -1 || kernel_id >= KT_COUNT) return fail(P3MZ_ERR_INVALID_ARG, "unknown kernel id");
  if (kernel_id >= 0 && ctx->kt_ev.empty()) {
    ctx->kt_ev.resize(2 * 2048);
    ctx->kt_bytes.resize(2048);
    for (hipEvent_t& e : ctx->kt_ev) P3MZ_HIP_TRY(hipEventCreate(&e));
  }
  ctx->kt_id = kernel_id;
  ctx->kt_used = 0;
  ctx->kt_total_ms = 0.0;
  ctx->kt_total_bytes = 0.0;
  ctx->kt_launches = 0;
  return P3MZ_OK;
}

p3mz_status p3mz_get_kernel_timer(const p3mz_ctx* ctx, double* total_ms, int64_t* launches, double* total_bytes) {
  if (!ctx || !total_ms || !launches || !total_bytes) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  *total_ms = ctx->kt_total_ms;
  *launches = ctx->kt_launches;
  *total_bytes = ctx->kt_total_bytes;
  return P3MZ_OK;
}

void p3mz_destroy(p3mz_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

const char* p3mz_status_string(p3mz_status s) {
  switch (s) {
    case P3MZ_OK: return "ok";
    case P3MZ_WARN_NOT_CONVERGED: return "warning: V-cycle cap reached before the tolerance";
    case P3MZ_ERR_INVALID_ARG: return "invalid argument";
    case P3MZ_ERR_NOT_NEUTRAL: return "system is not charge neutral";
    case P3MZ_ERR_MESH_SHAPE: return "unsupported mesh shape";
    case P3MZ_ERR_OUT_OF_MEMORY: return "out of device memory";
    case P3MZ_ERR_HIP: return "HIP runtime error";
    case P3MZ_ERR_NAN: return "non-finite position";
    case P3MZ_ERR_STATE: return "invalid state";
    case P3MZ_ERR_DENSITY: return "too many atoms in one bin";
  }
  return "unknown status";
}

const char* p3mz_last_error(void) { return g_last_error.c_str(); }

const char* p3mz_version(void) { return "p3maze-gfx950 0.1"; }

}  // extern "C"

// Host side of the library: planning, workspace allocation, the per-step
// launch sequence and the C ABI declared in include/p3maze.h.
#include <errno.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "kern.h"
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
  if (P.alpha * P.r_cut > 0.25 * kErfcMaxIntervals)
    return fail(P3MZ_ERR_INVALID_ARG, "alpha * r_cut must be <= 32 (the real-space term would vanish)");
  if (P.order < 2 || P.order > P3MZ_MAX_ORDER) return fail(P3MZ_ERR_INVALID_ARG, "order must be in 2..7");
  if (!(P.tol > 0) || P.tol_mode < 0 || P.tol_mode > 1) return fail(P3MZ_ERR_INVALID_ARG, "bad tolerance");
  if (P.max_cycles < 0 || P.max_cycles > P3MZ_MAX_CYCLES) return fail(P3MZ_ERR_INVALID_ARG, "max_cycles must be in 0..64");
  if (P.predictor < 0 || P.predictor > 3) return fail(P3MZ_ERR_INVALID_ARG, "predictor must be in 0..3");
  if (P.precision != P3MZ_PREC_FP64 && P.precision != P3MZ_PREC_MIXED && P.precision != P3MZ_PREC_MIXED32)
    return fail(P3MZ_ERR_INVALID_ARG, "bad precision");
  if (P.nu_pre < -1 || P.nu_post < -1 || P.nu_pre > 16 || P.nu_post > 16) return fail(P3MZ_ERR_INVALID_ARG, "bad sweep counts");
  if (P.excl_group < 0) return fail(P3MZ_ERR_INVALID_ARG, "excl_group must be >= 0");
  if (P.stencil < 0 || P.stencil > 1) return fail(P3MZ_ERR_INVALID_ARG, "stencil must be 0 or 1");
  if (P.stencil == 1 && P.order > 5) return fail(P3MZ_ERR_INVALID_ARG, "the fourth-order stencil needs order <= 5");
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
  // step weight nu <= 1/4; <= 1/6 for the fourth-order stencil, where the
  // K-step diffusion matches the Gaussian's fourth cumulant to O(h^4)
  pl->K = std::max(1, (int)ceil((P.stencil == 1 ? 3.0 : 2.0) * pl->sigma_s2 / (pl->h * pl->h)));
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

// Piecewise Chebyshev interpolant of erfcx(x) = exp(x^2) erfc(x) on [0, X]
// (intervals of width <= 1/4, degree kErfcDeg, values from long-double
// erfcl/expl at the Chebyshev nodes); the pair kernel forms
// erfc(x) = exp(-x^2) erfcx(x) from it.  Returns 0 intervals when X needs
// more than the kernel's table holds (parameters are validated against that).
int build_erfcx_table(double X, std::vector<double>* tab, double* scale) {
  int n = std::max(1, (int)ceil(X / 0.25));
  if (n > kErfcMaxIntervals) return 0;
  const double w = X / n;
  const int m = kErfcDeg + 1;
  tab->assign((size_t)n * m, 0.0);
  for (int i = 0; i < n; i++) {
    const long double a = (long double)i * w, b = a + w;
    long double f[kErfcDeg + 1];
    for (int k = 0; k < m; k++) {
      const long double th = (long double)M_PI * (k + 0.5L) / m;
      const long double x = 0.5L * (a + b) + 0.5L * (b - a) * cosl(th);
      f[k] = expl(x * x) * erfcl(x);
    }
    for (int j = 0; j < m; j++) {
      long double c = 0.0L;
      for (int k = 0; k < m; k++) c += f[k] * cosl((long double)M_PI * j * (k + 0.5L) / m);
      c *= 2.0L / m;
      if (j == 0) c *= 0.5L;
      (*tab)[(size_t)i * m + j] = (double)c;
    }
  }
  *scale = n / X;
  return n;
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

struct GraphSlot {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> key;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
};

struct p3mz_ctx {
  p3mz_params P{};
  Plan pl;
  int dev = 0;
  bool fp64 = true;
  bool src32 = false;      // charge assignment and smoothing in FP32
  size_t tsz = 8;
  int nu1 = 2, nu2 = 2;
  int smooth_tile = 0;     // smoothing launch shape (autotuned)
  int64_t n_atoms = 0;
  int64_t n3 = 0;
  double e_self = 0;
  int ntaps = 0, half = 0;
  // device buffers
  void* d_taps = nullptr;
  double* d_green = nullptr;
  double* d_qa = nullptr;
  int *d_key = nullptr, *d_slot = nullptr, *d_perm_raw = nullptr;
  void* d_rb = nullptr;   // int2 records in bin order: stencil origin, atom index
  void* d_rq = nullptr;   // double4 records in bin order: charge, fractional offsets
  int* d_cls = nullptr;   // first position of each crossing class in each bin (8 per bin)
  int ntx = 0, nbins = 0;
  int *d_count = nullptr, *d_start = nullptr, *d_bsum = nullptr;
  int nc = 1, ncells = 1;
  int ncells_max = 1;     // cell arrays are sized for the cells of edge r_cut
  // neighbour lists (skin 0: none, the pair kernels scan the cells every step)
  double nbr_skin = 0.0;
  int nbr_cap = 0;
  int* d_nbr = nullptr;     // [n_atoms][nbr_cap] entries
  int* d_nlist = nullptr;   // entries per atom
  double* d_ref = nullptr;  // {x, y, z, q} of each atom at the last build (cell order)
  int *d_ckey = nullptr, *d_cslot = nullptr, *d_ccount = nullptr, *d_cstart = nullptr, *d_cperm_raw = nullptr,
      *d_cperm = nullptr;
  double* d_spos = nullptr;   // cell-ordered {x, y, z, q} for the pair kernels
  double* d_erfc = nullptr;   // erfcx table of the pair kernel
  int erfc_n = 0;
  double erfc_scale = 0.0;
  double *d_q = nullptr, *d_qs = nullptr, *d_tmp = nullptr;
  double* d_sigma = nullptr;
  double* d_y[2] = {nullptr, nullptr};   // multiplier ping-pong (the control block's final_buf names the last)
  double* d_phi[2] = {nullptr, nullptr};
  double* d_yh[3] = {nullptr, nullptr, nullptr};
  float* d_phi32 = nullptr;
  LevelBufs lv[P3MZ_MAX_LEVELS];
  double* d_partial = nullptr;
  double* d_spart = nullptr;     // sigma's partials when the first outer residual reduces them
  double* d_nfpart = nullptr;    // net-force partials of the pair kernels
  double* d_nepart = nullptr;    // energy partials of the MD pair and bonded terms
  Ctl* d_ctl = nullptr;
  Ctl* h_ctl = nullptr;         // pinned mirror
  double* d_energy = nullptr;   // internal energy4 when the caller passes none
  // md
  double th_gamma = 0.0, th_kt = 0.0;   // OVRVO thermostat (gamma 0: none)
  uint64_t th_seed = 0;
  double* d_md_force = nullptr;
  double* d_e_other = nullptr;
  bool md_have_force = false;
  std::vector<uint64_t> md_force_key;   // buffers and terms d_md_force was computed with
  // host mirror of the device history state (refreshed after every step)
  Ctl mirror{};
  int last_cycles = 0;
  p3mz_stats st{};
  std::vector<void*> allocs;
  // graphs: captured on a private stream, launched on the caller's stream
  bool use_graphs = true;
  bool capturing = false;        // enqueueing into a graph capture right now
  bool sub_events = false;       // the sub-stage events were recorded this step
  bool ran_graphs = false;       // the last step was launched from graphs
  hipStream_t cap = nullptr;
  GraphSlot g_pre, g_post1, g_post2, g_md_post2;
  // g_cycles[k]: k consecutive V-cycles (each with its outer residual) in one graph
  static constexpr int kCycleGraphMax = 16;
  GraphSlot g_cycles[kCycleGraphMax + 1];
  // optional timing: stage events and one kernel family's per-launch events
  bool timing = false;
  hipEvent_t stage_ev[5] = {};
  int kt_id = -1;
  std::vector<hipEvent_t> kt_ev;
  std::vector<double> kt_bytes;
  int kt_used = 0;
  double kt_total_ms = 0.0, kt_total_bytes = 0.0;
  int64_t kt_launches = 0;
  static constexpr size_t kKtKeep = 65536;   // per-launch records kept for p3mz_get_kernel_launches
  std::vector<float> kt_hist_ms;
  std::vector<double> kt_hist_bytes;

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
  void release(void* p) {
    if (!p) return;
    for (size_t k = 0; k < allocs.size(); k++)
      if (allocs[k] == p) {
        (void)hipFree(p);
        allocs.erase(allocs.begin() + (long)k);
        return;
      }
  }
  void drop_graphs() {
    g_pre.reset();
    for (GraphSlot& g : g_cycles) g.reset();
    g_post1.reset();
    g_post2.reset();
    g_md_post2.reset();
  }
  ~p3mz_ctx() {
    drop_graphs();
    for (void* v : allocs) (void)hipFree(v);
    if (h_ctl) (void)hipHostFree(h_ctl);
    for (hipEvent_t e : stage_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : kt_ev) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// The context whose work is being enqueued (kernel-timer hooks read it).
static p3mz_ctx* g_active = nullptr;

thread_local Recorder* g_recorder = nullptr;

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

uint64_t bits(double v) {
  uint64_t u;
  memcpy(&u, &v, 8);
  return u;
}

// ---------------------------------------------------------------------------
// Tuning cache: one JSON object per line inside an "entries" array, keyed by
// device, mesh edge, assignment order and precision.  Written by
// p3mz_autotune, read when a context asks for the tuned sweep counts.
// ---------------------------------------------------------------------------
struct TuneEntry {
  int nu_pre = 2, nu_post = 2, smooth_tile = 0;
  double ms = 0.0;
};

std::string tune_path() {
  const char* e = getenv("P3MZ_TUNE_CACHE");
  if (e && *e) return e;
  const char* home = getenv("HOME");
  return std::string(home && *home ? home : "/tmp") + "/.cache/p3maze/tune.json";
}

std::string tune_key(int n, int p, int precision) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == '"' || ch == ' ') ch = '_';
  char buf[256];
  snprintf(buf, sizeof buf, "%s/n%d/p%d/%s", arch.c_str(), n, p,
           precision == P3MZ_PREC_FP64 ? "fp64" : precision == P3MZ_PREC_MIXED ? "mixed" : "mixed32");
  return buf;
}

// All entries of the cache file (key -> entry); a missing file is empty.
std::vector<std::pair<std::string, TuneEntry>> tune_read() {
  std::vector<std::pair<std::string, TuneEntry>> out;
  FILE* f = fopen(tune_path().c_str(), "r");
  if (!f) return out;
  char line[1024], key[512];
  while (fgets(line, sizeof line, f)) {
    TuneEntry t;
    if (sscanf(line, " {\"key\": \"%511[^\"]\", \"nu_pre\": %d, \"nu_post\": %d, \"smooth_tile\": %d, \"ms\": %lf",
               key, &t.nu_pre, &t.nu_post, &t.smooth_tile, &t.ms) == 5)
      out.emplace_back(key, t);
  }
  fclose(f);
  return out;
}

bool tune_lookup(const std::string& key, TuneEntry* t) {
  for (auto& kv : tune_read())
    if (kv.first == key) {
      *t = kv.second;
      return true;
    }
  return false;
}

p3mz_status tune_store(const std::string& key, const TuneEntry& t) {
  auto all = tune_read();
  bool found = false;
  for (auto& kv : all)
    if (kv.first == key) {
      kv.second = t;
      found = true;
    }
  if (!found) all.emplace_back(key, t);
  const std::string path = tune_path();
  // create the parent directories
  for (size_t i = 1; i < path.size(); i++)
    if (path[i] == '/') {
      const std::string d = path.substr(0, i);
      if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST)
        return fail(P3MZ_ERR_INVALID_ARG, "cannot create the tuning cache directory " + d);
    }
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return fail(P3MZ_ERR_INVALID_ARG, "cannot write the tuning cache " + tmp);
  fprintf(f, "{\"entries\": [\n");
  for (size_t i = 0; i < all.size(); i++)
    fprintf(f, "  {\"key\": \"%s\", \"nu_pre\": %d, \"nu_post\": %d, \"smooth_tile\": %d, \"ms\": %.6f}%s\n",
            all[i].first.c_str(), all[i].second.nu_pre, all[i].second.nu_post, all[i].second.smooth_tile,
            all[i].second.ms, i + 1 < all.size() ? "," : "");
  fprintf(f, "]}\n");
  if (fclose(f) != 0 || rename(tmp.c_str(), path.c_str()) != 0)
    return fail(P3MZ_ERR_INVALID_ARG, "cannot write the tuning cache " + path);
  return P3MZ_OK;
}

// Cells per box edge for a cell list of cells at least `width` wide (fewer
// than 3: one cell, every pair is a candidate).
int cells_per_edge(double box, double width) {
  int nc = (int)floor(box / width);
  if (nc < 3) nc = 1;
  if (nc > 256) nc = 256;
  return nc;
}

// Default skin of the neighbour lists, as a fraction of r_cut.
constexpr double kSkinFraction = 0.1;

// Neighbour lists of skin `skin` (0: none) and `cap` entries per atom (0:
// from the mean density, 30 % above the expected count plus 64).  The cell
// list is rebuilt for cells at least r_cut + skin wide; the first step
// after this builds the lists.
p3mz_status nbr_configure(p3mz_ctx* c, double skin, int cap) {
  c->release(c->d_nbr);
  c->release(c->d_nlist);
  c->release(c->d_ref);
  c->d_nbr = c->d_nlist = nullptr;
  c->d_ref = nullptr;
  c->nbr_skin = 0.0;
  c->nbr_cap = 0;
  c->drop_graphs();
  // without lists until the new ones are in place: a failure below leaves
  // the context scanning cells of edge r_cut
  c->nc = cells_per_edge(c->P.box, c->P.r_cut);
  c->ncells = c->nc * c->nc * c->nc;
  if (skin <= 0.0) return P3MZ_OK;
  const double rl = c->P.r_cut + skin;
  const int64_t na = c->n_atoms;
  if (cap <= 0) {
    const double expect = 4.0 / 3.0 * kPi * rl * rl * rl * (double)na / (c->P.box * c->P.box * c->P.box);
    cap = (int)std::min<double>(1.3 * expect + 64.0, (double)(1 << 24));
  }
  cap = (int)std::min<int64_t>((cap + 63) / 64 * 64, (std::max<int64_t>(na - 1, 1) + 63) / 64 * 64);
  int *nbr = nullptr, *nlist = nullptr;
  double* ref = nullptr;
  p3mz_status st = c->alloc(&nbr, (size_t)na * cap);
  if (st == P3MZ_OK) st = c->alloc(&nlist, (size_t)na);
  if (st == P3MZ_OK) st = c->alloc(&ref, 4 * (size_t)na);
  hipError_t e = hipSuccess;
  const int one = 1;
  // NaN reference positions: the first check flags a build
  if (st == P3MZ_OK) e = hipMemset(ref, 0xff, sizeof(double) * 4 * (size_t)na);
  if (st == P3MZ_OK && e == hipSuccess) e = hipMemcpy(&c->d_ctl->nbr_stale, &one, sizeof(int), hipMemcpyHostToDevice);
  if (st != P3MZ_OK || e != hipSuccess) {
    c->release(nbr);
    c->release(nlist);
    c->release(ref);
    return st != P3MZ_OK ? st : hip_fail(e, "neighbour-list set-up", __FILE__, __LINE__);
  }
  c->nc = cells_per_edge(c->P.box, rl);
  c->ncells = c->nc * c->nc * c->nc;
  c->d_nbr = nbr;
  c->d_nlist = nlist;
  c->d_ref = ref;
  c->nbr_skin = skin;
  c->nbr_cap = cap;
  return P3MZ_OK;
}

p3mz_status setup(p3mz_ctx* c, const double* charges_host) {
  const Plan& pl = c->pl;
  const int n = pl.n;
  c->n3 = (int64_t)n * n * n;
  c->fp64 = c->P.precision == P3MZ_PREC_FP64;
  c->src32 = c->P.precision == P3MZ_PREC_MIXED32;
  c->tsz = c->fp64 ? 8 : 4;
  TuneEntry tuned;
  const bool have_tune = tune_lookup(tune_key(pl.n, pl.p, c->P.precision), &tuned);
  c->nu1 = c->P.nu_pre >= 0 ? c->P.nu_pre : (have_tune ? tuned.nu_pre : 2);
  c->nu2 = c->P.nu_post >= 0 ? c->P.nu_post : (have_tune ? tuned.nu_post : 2);
  if (c->nu1 + c->nu2 < 1) return fail(P3MZ_ERR_INVALID_ARG, "nu_pre + nu_post must be >= 1");
  P3MZ_HIP_TRY(hipGetDevice(&c->dev));
  P3MZ_HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  double e_self = 0.0;
  for (int64_t a = 0; a < c->n_atoms; a++) e_self -= c->P.coulomb_k * c->P.alpha / sqrt(kPi) * charges_host[a] * charges_host[a];
  c->e_self = e_self;
  P3MZ_TRY(c->alloc(&c->d_qa, c->n_atoms));
  P3MZ_HIP_TRY(hipMemcpy(c->d_qa, charges_host, sizeof(double) * c->n_atoms, hipMemcpyHostToDevice));
  // The charge source (spread, smoothing) is FP64 in the FP64 and MIXED
  // modes and FP32 in MIXED32; sigma_p is formed in FP64 in every mode.
  std::vector<double> taps;
  smoothing_taps(n, pl.K, pl.nu_s, &taps, &c->half);
  c->ntaps = (int)taps.size();
  // the launch shape never changes results, so a tuned one is always taken;
  // otherwise the first shape (in preference order) that fits the mesh
  c->smooth_tile = have_tune && smooth_tile_ok(tuned.smooth_tile, n, c->ntaps) ? tuned.smooth_tile : -1;
  for (int t = 0; c->smooth_tile < 0 && t < smooth_tile_count(); t++)
    if (smooth_tile_ok(t, n, c->ntaps)) c->smooth_tile = t;
  if (c->smooth_tile < 0) return fail(P3MZ_ERR_MESH_SHAPE, "no smoothing launch shape fits this mesh");
  P3MZ_TRY(c->allocb(&c->d_taps, taps.size() * 8));
  if (c->src32) {
    std::vector<float> t32(taps.begin(), taps.end());
    P3MZ_HIP_TRY(hipMemcpy(c->d_taps, t32.data(), t32.size() * 4, hipMemcpyHostToDevice));
  } else {
    P3MZ_HIP_TRY(hipMemcpy(c->d_taps, taps.data(), taps.size() * 8, hipMemcpyHostToDevice));
  }
  double g[64];
  coarse_green(g);
  P3MZ_TRY(c->alloc(&c->d_green, 64));
  P3MZ_HIP_TRY(hipMemcpy(c->d_green, g, sizeof g, hipMemcpyHostToDevice));
  const int64_t na = c->n_atoms;
  c->ntx = n / kTile;
  c->nbins = c->ntx * c->ntx * c->ntx;
  P3MZ_TRY(c->allocb(&c->d_rb, (size_t)na * 8));
  P3MZ_TRY(c->allocb(&c->d_rq, (size_t)na * 32));
  P3MZ_TRY(c->alloc(&c->d_key, na));
  P3MZ_TRY(c->alloc(&c->d_slot, na));
  P3MZ_TRY(c->alloc(&c->d_perm_raw, na));
  P3MZ_TRY(c->alloc(&c->d_count, c->nbins));
  P3MZ_TRY(c->alloc(&c->d_start, c->nbins + 1));
  P3MZ_TRY(c->alloc(&c->d_cls, 8 * (size_t)c->nbins));
  P3MZ_HIP_TRY(hipMemset(c->d_count, 0, sizeof(int) * c->nbins));
  c->nc = cells_per_edge(c->P.box, c->P.r_cut);
  c->ncells = c->ncells_max = c->nc * c->nc * c->nc;
  P3MZ_TRY(c->alloc(&c->d_ckey, na));
  P3MZ_TRY(c->alloc(&c->d_cslot, na));
  P3MZ_TRY(c->alloc(&c->d_cperm_raw, na));
  P3MZ_TRY(c->alloc(&c->d_cperm, na));
  {
    // a valid permutation before the first cell sort (the neighbour check
    // reads the order of the last build)
    std::vector<int> id((size_t)na);
    for (int64_t a = 0; a < na; a++) id[(size_t)a] = (int)a;
    P3MZ_HIP_TRY(hipMemcpy(c->d_cperm, id.data(), sizeof(int) * (size_t)na, hipMemcpyHostToDevice));
  }
  P3MZ_TRY(c->alloc(&c->d_spos, 4 * na));
  {
    std::vector<double> tab;
    c->erfc_n = build_erfcx_table(c->P.alpha * c->P.r_cut, &tab, &c->erfc_scale);
    P3MZ_TRY(c->alloc(&c->d_erfc, std::max<size_t>(tab.size(), 1)));
    if (!tab.empty()) P3MZ_HIP_TRY(hipMemcpy(c->d_erfc, tab.data(), tab.size() * 8, hipMemcpyHostToDevice));
  }
  P3MZ_TRY(c->alloc(&c->d_ccount, c->ncells));
  P3MZ_TRY(c->alloc(&c->d_cstart, c->ncells + 1));
  P3MZ_HIP_TRY(hipMemset(c->d_ccount, 0, sizeof(int) * c->ncells));
  P3MZ_TRY(c->alloc(&c->d_bsum, std::max(scan_partials(c->nbins), scan_partials(c->ncells))));
  const size_t n3 = (size_t)c->n3;
  P3MZ_TRY(c->alloc(&c->d_q, n3));
  P3MZ_TRY(c->alloc(&c->d_qs, n3));
  P3MZ_TRY(c->alloc(&c->d_tmp, n3));
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
    if (l < pl.tail && nl <= kFusedEdgeMax && nl >= 16) {
      P3MZ_TRY(c->allocb(&b.d0, half * c->tsz));
      P3MZ_TRY(c->allocb(&b.d1, half * c->tsz));
      b.fty = b.ftz = fused_tile(nl);
    }
    if (l < pl.tail && (nl == 512 || nl == 256) && !c->fp64) {   // output of the fused post-smoothing
      P3MZ_TRY(c->allocb(&b.s0, half * c->tsz));
      P3MZ_TRY(c->allocb(&b.s1, half * c->tsz));
    }
  }
  // every reduction grid is capped, so one fixed-size partial buffer fits all
  P3MZ_TRY(c->alloc(&c->d_partial, kPartialSlots));
  P3MZ_TRY(c->alloc(&c->d_spart, kPartialSlots));
  P3MZ_TRY(c->alloc(&c->d_nfpart, 3 * kPartialSlots));
  P3MZ_TRY(c->alloc(&c->d_nepart, 2 * kPartialSlots));
  P3MZ_TRY(c->alloc(&c->d_ctl, 1));
  P3MZ_HIP_TRY(hipHostMalloc((void**)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  memset(&c->mirror, 0, sizeof(Ctl));
  c->mirror.cold = 1;
  c->mirror.yh0 = 0;
  c->mirror.yh1 = 1;
  c->mirror.yh2 = 2;
  c->mirror.predictor = c->P.predictor;
  P3MZ_HIP_TRY(hipMemcpy(c->d_ctl, &c->mirror, sizeof(Ctl), hipMemcpyHostToDevice));
  P3MZ_TRY(c->alloc(&c->d_energy, 4));
  P3MZ_TRY(c->alloc(&c->d_md_force, 3 * na));
  P3MZ_TRY(c->alloc(&c->d_e_other, 1));
  size_t lds = 0;
  P3MZ_HIP_TRY(tail_configure(c->fp64, n >> pl.tail, pl.levels - pl.tail, &lds));
  P3MZ_HIP_TRY(smooth_configure());
  P3MZ_HIP_TRY(fused_configure());
  P3MZ_TRY(nbr_configure(c, kSkinFraction * c->P.r_cut, 0));
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  return P3MZ_OK;
}

// ---------------------------------------------------------------------------
// The step, as three launch sequences.  Each is enqueued either directly
// (eager) or once into a captured graph that is replayed every step.
// ---------------------------------------------------------------------------
// Stage events are recorded only on the caller's stream between graph
// launches (events recorded inside a graph cannot be timed); the sub-stage
// boundaries 1 and 2 exist only when the step is launched kernel by kernel.
void stage(p3mz_ctx* c, int i, hipStream_t s) {
  if (!c->timing || c->capturing) return;
  (void)hipEventRecord(c->stage_ev[i], s);
  if (i == 1 || i == 2) c->sub_events = true;
}

// bin + deterministic order, spread, smoothing, sigma_p and predictor, first residual
p3mz_status enq_pre(p3mz_ctx* c, const double* pos, hipStream_t s) {
  const Plan& pl = c->pl;
  const int n = pl.n, na = (int)c->n_atoms;
  const double N3 = (double)c->n3, ts = (double)c->tsz;
  rec_key(100);
  P3MZ_HIP_TRY(launch_bin_tiles(na, pos, c->P.box, n, pl.p, kTile, c->ntx, c->d_key, c->d_slot, c->d_count, c->d_ctl,
                                s));
  rec_key(101);
  P3MZ_HIP_TRY(launch_scan(c->nbins, c->d_count, c->d_start, c->d_bsum, s));
  rec_key(102);
  P3MZ_HIP_TRY(launch_scatter(na, c->d_key, c->d_slot, c->d_start, c->d_perm_raw, s));
  rec_key(103);
  P3MZ_HIP_TRY(launch_sort_pack(c->nbins, c->d_start, c->d_perm_raw, na, pos, c->d_qa, c->P.box, n, pl.p, kTile,
                                c->d_rb, c->d_rq, c->d_cls, s));
  rec_key(104);
  kt_begin(KT_SPREAD, 0, s);
  const double qsz = c->src32 ? 4.0 : 8.0;   // bytes per point of the charge source
  P3MZ_HIP_TRY(launch_spread(!c->src32, n, pl.p, kTile, c->ntx, c->P.box, c->d_start, c->d_cls, c->d_rb, c->d_rq,
                             c->d_q, s));
  // algorithmic bytes: the mesh written once, each atom's 40-byte record read once
  kt_end(KT_SPREAD, 0, qsz * N3 + 40.0 * (double)na, s);
  double* src[3] = {c->d_q, c->d_qs, c->d_tmp};
  double* dst[3] = {c->d_qs, c->d_tmp, c->d_qs};
  for (int axis = 0; axis < 3; axis++) {
    rec_key(105 + axis);
    kt_begin(KT_SMOOTH, 0, s);
    P3MZ_HIP_TRY(launch_smooth(!c->src32, n, axis, c->smooth_tile, c->ntaps, c->half, c->d_taps, src[axis], dst[axis],
                               s));
    kt_end(KT_SMOOTH, 0, 2.0 * qsz * N3, s);
  }
  stage(c, 1, s);
  rec_key(110);
  kt_begin(KT_SIGMA, 0, s);
  // A single system folds the sigma pass's reduction into the first outer
  // residual (every workgroup reduces sigma's partials, kept in a buffer of
  // their own) and leaves that residual's stop decision to the first
  // cycle's tail: two launches less per step.  A batch keeps both passes.
  const bool fold = !g_recorder;
  P3MZ_HIP_TRY(launch_sigma(n, pl.h, c->src32, c->d_qs, c->d_phi[0], c->d_phi[1], c->d_yh[0], c->d_yh[1], c->d_yh[2],
                            c->d_sigma, c->d_y[0], c->P.tol, c->P.tol_mode, fold ? c->d_spart : c->d_partial,
                            c->d_ctl, s, !fold, c->P.stencil));
  kt_end(KT_SIGMA, 0, (56.0 + qsz) * N3, s);
  const LevelBufs& f = c->lv[0];
  rec_key(111);
  kt_begin(KT_OUTER, 0, s);
  P3MZ_HIP_TRY(launch_outer(c->fp64, n, 1, c->P.max_cycles, c->d_sigma, c->d_y[0], c->d_y[1], f.e0, f.e1, f.r0, f.r1,
                            c->d_partial, c->d_ctl, s, !fold, fold ? c->d_spart : nullptr, c->P.tol,
                            c->P.tol_mode, c->P.stencil));
  kt_end(KT_OUTER, 0, (16.0 + ts) * N3, s);
  return P3MZ_OK;
}

// one V-cycle and the following outer residual
p3mz_status enq_cycle(p3mz_ctx* c, hipStream_t s) {
  const Plan& pl = c->pl;
  const LevelBufs& f = c->lv[0];
  const double N3 = (double)c->n3, ts = (double)c->tsz;
  // A single system: the tail makes the stop decision of the previous outer
  // residual, and this cycle's is made by the next cycle's tail or ahead of
  // the field update (one launch less per cycle).  A batch decides right
  // after each residual: its systems converge at different cycles, and a
  // deferred decision would let the converged ones run the next cycle's
  // upper levels.
  const bool defer = !g_recorder;
  const Decide d{c->d_partial, red_blocks((int64_t)c->n3 / 4), (int)c->n3, c->P.max_cycles};
  P3MZ_HIP_TRY(launch_vcycle(c->fp64, c->lv, pl.levels, pl.tail, c->nu1, c->nu2, c->d_green, c->d_ctl, s,
                             defer ? &d : nullptr));
  rec_key(4100);
  kt_begin(KT_OUTER, 0, s);
  P3MZ_HIP_TRY(launch_outer(c->fp64, pl.n, 0, c->P.max_cycles, c->d_sigma, c->d_y[0], c->d_y[1],
                            cycle_e0(f, c->fp64, c->nu2), cycle_e1(f, c->fp64, c->nu2), f.r0,
                            f.r1, c->d_partial, c->d_ctl, s, !defer, nullptr, 0.0, 0, c->P.stencil));
  kt_end(KT_OUTER, 0, (24.0 + 2.0 * ts) * N3, s);
  return P3MZ_OK;
}

// field update and gather on the new potential
p3mz_status enq_post1(p3mz_ctx* c, double* force, hipStream_t s) {
  const Plan& pl = c->pl;
  const int n = pl.n, na = (int)c->n_atoms;
  const double N3 = (double)c->n3;
  // a single system's last stop decision is made by every workgroup of the
  // field update (a batch made it right after the residual)
  const Decide d{c->d_partial, red_blocks((int64_t)c->n3 / 4), (int)c->n3, c->P.max_cycles};
  rec_key(5000);
  kt_begin(KT_PHI, 0, s);
  P3MZ_HIP_TRY(launch_phi_update(n, pl.h, c->d_phi[0], c->d_phi[1], c->d_y[0], c->d_y[1], c->d_yh[0], c->d_yh[1],
                                 c->d_yh[2], c->d_phi32, c->d_ctl, s, g_recorder ? nullptr : &d));
  kt_end(KT_PHI, 0, 40.0 * N3 + (c->fp64 ? 0.0 : 4.0 * N3), s);
  stage(c, 2, s);
  rec_key(5001);
  kt_begin(KT_GATHER, 0, s);
  P3MZ_HIP_TRY(launch_gather(c->fp64, na, n, pl.p, kTile, c->ntx, pl.h, c->P.coulomb_k, c->d_start, c->d_rb, c->d_rq,
                             c->d_phi[0], c->d_phi[1], c->d_phi32, force, c->d_partial, c->d_ctl, s, true,
                             c->P.stencil));
  // algorithmic bytes: the potential once, plus each atom's 40-byte record
  // and its force (the (p+2)^3 neighbourhood reads are shared by atoms)
  kt_end(KT_GATHER, 0, N3 * (c->fp64 ? 8.0 : 4.0) + (double)na * 64.0, s);
  return P3MZ_OK;
}

// short-range pairs on a fresh cell list, energies, history rotation
// With neighbour lists the cell list and the lists are rebuilt only on the
// steps the check flags (the rebuild launches test the flag on the device).
// ne (MD steps): the list pass of the pair kernel also adds the MD pair term
// of model ne->model; *ne_written gets the number of its energy partials.
struct NePair {
  int model;
  double p0, p1;
};
p3mz_status enq_post2(p3mz_ctx* c, const double* pos, double* force, double* energy, hipStream_t s,
                      const NePair* ne = nullptr, int* ne_written = nullptr) {
  const int na = (int)c->n_atoms;
  const bool nbr = c->d_nbr != nullptr;
  const int* gate = nbr ? &c->d_ctl->nbr_stale : nullptr;
  if (nbr)
    P3MZ_HIP_TRY(launch_nbr_check(na, c->P.box, c->nbr_skin, c->d_cperm, pos, c->d_qa, c->d_spos, c->d_ref, c->d_ctl,
                                  s));
  rec_key(6000);
  P3MZ_HIP_TRY(launch_bin_cells(na, pos, c->P.box, c->nc, c->d_ckey, c->d_cslot, c->d_ccount, c->d_ctl, s, gate));
  rec_key(6001);
  P3MZ_HIP_TRY(launch_scan(c->ncells, c->d_ccount, c->d_cstart, c->d_bsum, s, gate));
  rec_key(6002);
  P3MZ_HIP_TRY(launch_scatter(na, c->d_ckey, c->d_cslot, c->d_cstart, c->d_cperm_raw, s, gate));
  rec_key(6003);
  P3MZ_HIP_TRY(launch_sort_bins(c->ncells, c->d_cstart, c->d_cperm_raw, c->d_cperm, c->d_ctl, s, gate));
  P3MZ_HIP_TRY(launch_cell_pack(na, c->d_cperm, pos, c->d_qa, c->d_spos, s, gate));
  if (nbr)
    P3MZ_HIP_TRY(launch_nbr_build(na, c->P.box, c->P.r_cut + c->nbr_skin, c->nc, c->P.excl_group, c->nbr_cap,
                                  c->d_cstart, c->d_cperm, c->d_spos, c->d_ref, c->d_nbr, c->d_nlist, c->d_ctl, s));
  rec_key(6004);
  kt_begin(KT_SR, 0, s);
  P3MZ_HIP_TRY(launch_sr(na, pos, c->d_qa, c->P.box, c->P.alpha, c->P.r_cut, c->P.coulomb_k, c->nc, c->P.excl_group,
                         c->d_cstart, c->d_cperm, c->d_spos, c->d_erfc, c->erfc_n, c->erfc_scale, force, c->e_self,
                         energy ? energy : c->d_energy,
                         c->d_partial, c->d_nfpart, c->d_ctl, s, c->d_nbr, c->d_nlist, c->nbr_cap,
                         ne && c->d_nbr ? ne->model : 0, ne ? ne->p0 : 0.0, ne ? ne->p1 : 0.0, c->d_nepart,
                         ne_written));
  kt_end(KT_SR, 0, (double)na * 56.0, s);
  rec_key(6005);
  P3MZ_HIP_TRY(launch_advance(c->d_ctl, s));
  return P3MZ_OK;
}

struct MdArgs {
  double *pos, *vel, *elog;
  const double* mass;
  int* clog;
  double dt, f2a, mv2e, p[6];
  int model;
  Thermostat th;
};

// the rest of an MD step after the mesh step: pairs, non-electrostatic
// terms, closing half-kick and the energy log
p3mz_status enq_md_post2(p3mz_ctx* c, const MdArgs& m, hipStream_t s) {
  const int na = (int)c->n_atoms;
  // with neighbour lists, the pair term of the model rides along the
  // short-range list pass; the non-electrostatic kernel then covers only
  // the atoms over the list capacity (and the bonded terms)
  const NePair ne{m.model, m.p[0], m.p[1]};
  int prior = 0;
  P3MZ_TRY(enq_post2(c, m.pos, c->d_md_force, c->d_energy, s, m.model != 0 ? &ne : nullptr, &prior));
  // the cell list of the short-range pass is still valid for these positions
  rec_key(6100);
  P3MZ_HIP_TRY(launch_nonelec(na, m.pos, c->P.box, c->P.r_cut, m.model, m.p[0], m.p[1], m.p[2], m.p[3], m.p[4],
                              m.p[5], c->nc, c->d_cstart, c->d_cperm, c->d_spos, c->d_md_force, c->d_nepart,
                              c->d_e_other, s, c->d_nbr, c->d_nlist, c->nbr_cap, prior, prior > 0));
  rec_key(6101);
  P3MZ_HIP_TRY(launch_kick_drift(na, m.pos, m.vel, c->d_md_force, m.mass, m.dt, m.f2a, 0, s, &m.th));
  rec_key(6102);
  P3MZ_HIP_TRY(launch_kinetic_log(na, m.vel, m.mass, m.mv2e, c->d_energy, c->d_e_other, m.elog, m.clog, c->d_ctl,
                                  c->d_partial, s));
  return P3MZ_OK;
}

// Enqueue `body` on s: eagerly, or through the graph in `slot` (captured on
// the private stream when the key changes).  A failed capture switches the
// context to eager launches for good.
template <typename F>
p3mz_status run_seq(p3mz_ctx* c, GraphSlot& slot, const std::vector<uint64_t>& key, hipStream_t s, F body) {
  if (!c->use_graphs || c->kt_id >= 0) return body(s);
  if (!slot.exec || slot.key != key) {
    slot.reset();
    P3MZ_HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    p3mz_status st = body(c->cap);
    c->capturing = false;
    hipError_t e = hipStreamEndCapture(c->cap, &slot.graph);
    if (st != P3MZ_OK || e != hipSuccess) {
      slot.reset();
      (void)hipGetLastError();
      c->use_graphs = false;
      return body(s);
    }
    e = hipGraphInstantiate(&slot.exec, slot.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      slot.reset();
      (void)hipGetLastError();
      c->use_graphs = false;
      return body(s);
    }
    slot.key = key;
  }
  P3MZ_HIP_TRY(hipGraphLaunch(slot.exec, s));
  c->ran_graphs = true;
  return P3MZ_OK;
}

// Copies the head of the control block (done, cycles, status, final_buf,
// nan_flag) to the pinned mirror and waits for it.
p3mz_status read_head(p3mz_ctx* c, hipStream_t s) {
  P3MZ_HIP_TRY(hipMemcpyAsync(c->h_ctl, c->d_ctl, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
  P3MZ_HIP_TRY(hipStreamSynchronize(s));
  return P3MZ_OK;
}

// V-cycles, then the field update and gather (post1): the expected number
// of cycles (the last step's count) is enqueued at once and post1 right
// behind it, so a correct guess costs no host round trip inside the mesh
// step; post1's kernels do nothing unless the solve has converged.  The
// device flag is read after post1; if the solve is still open, cycles follow
// one at a time, each followed by post1 again.  Returns with the head of the
// control block read after the last post1.
p3mz_status run_solve(p3mz_ctx* c, double* force, hipStream_t s) {
  int issued = 0;
  int batch = std::max(1, c->last_cycles);
  for (;;) {
    // the cycles of a batch go out as few graph launches as possible
    for (int left = std::min(batch, c->P.max_cycles - issued); left > 0;) {
      const int k = std::min(left, p3mz_ctx::kCycleGraphMax);
      P3MZ_TRY(run_seq(c, c->g_cycles[k], {(uint64_t)k}, s, [&](hipStream_t q) {
        for (int i = 0; i < k; i++) P3MZ_TRY(enq_cycle(c, q));
        return P3MZ_OK;
      }));
      left -= k;
      issued += k;
    }
    P3MZ_TRY(run_seq(c, c->g_post1, {(uint64_t)(uintptr_t)force, c->timing}, s,
                     [&](hipStream_t q) { return enq_post1(c, force, q); }));
    stage(c, 3, s);
    P3MZ_TRY(read_head(c, s));
    if (c->h_ctl->done || c->h_ctl->nan_flag || issued >= c->P.max_cycles) return P3MZ_OK;
    batch = 1;
  }
}

p3mz_status on_nan(p3mz_ctx* c) {
  // drop the history: the next step is a cold solve
  P3MZ_HIP_TRY(hipMemcpy(&c->mirror, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  c->mirror.nan_flag = 0;
  c->mirror.cold = 1;
  c->mirror.n_yh = 0;
  c->mirror.m_eff = 0;
  P3MZ_HIP_TRY(hipMemcpy(c->d_ctl, &c->mirror, sizeof(Ctl), hipMemcpyHostToDevice));
  c->last_cycles = 0;
  c->md_have_force = false;
  return fail(P3MZ_ERR_NAN, "non-finite position");
}

// After the post sequence: read the whole control block and fill the stats.
p3mz_status finish(p3mz_ctx* c, hipStream_t s) {
  P3MZ_HIP_TRY(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  P3MZ_HIP_TRY(hipStreamSynchronize(s));
  const Ctl& h = *c->h_ctl;
  const int was_cold = c->mirror.cold, m_eff = c->mirror.m_eff;
  c->mirror = h;
  c->last_cycles = h.cycles;
  p3mz_stats& st = c->st;
  st.status = h.status ? P3MZ_WARN_NOT_CONVERGED : P3MZ_OK;
  st.cycles = h.cycles;
  st.cold = was_cold;
  st.m_eff = m_eff;
  st.nu_pre = c->nu1;
  st.nu_post = c->nu2;
  st.K = c->pl.K;
  st.levels = c->pl.levels;
  st.nu_smooth = c->pl.nu_s;
  st.thresh = h.thresh;
  st.norm_qs = h.norm_qs;
  for (int i = 0; i <= P3MZ_MAX_CYCLES; i++) st.res_hist[i] = i <= h.cycles ? h.res_hist[i] : 0.0;
  st.e_sr = h.e_sr;
  st.e_lr = h.e_lr;
  st.e_self = c->e_self;
  st.e_total = h.e_sr + h.e_lr + c->e_self;
  st.steps = h.steps;
  st.graphs = c->ran_graphs;
  for (int k = 0; k < 3; k++) st.net_force[k] = h.net_force[k];
  if (c->timing) {
    float ms = 0.f;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->stage_ev[0], c->stage_ev[3]));
    st.ms_mesh = ms;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->stage_ev[3], c->stage_ev[4]));
    st.ms_short_range = ms;
    st.ms_spread = st.ms_solve = st.ms_gather = -1.0;
    if (c->sub_events) {
      P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->stage_ev[0], c->stage_ev[1]));
      st.ms_spread = ms;
      P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->stage_ev[1], c->stage_ev[2]));
      st.ms_solve = ms;
      P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->stage_ev[2], c->stage_ev[3]));
      st.ms_gather = ms;
    }
  }
  for (int i = 0; i + 1 < c->kt_used; i += 2) {
    float ms = 0.f;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, c->kt_ev[i], c->kt_ev[i + 1]));
    c->kt_total_ms += ms;
    c->kt_total_bytes += c->kt_bytes[i / 2];
    c->kt_launches++;
    if (c->kt_hist_ms.size() < p3mz_ctx::kKtKeep) {
      c->kt_hist_ms.push_back(ms);
      c->kt_hist_bytes.push_back(c->kt_bytes[i / 2]);
    }
  }
  c->kt_used = 0;
  return P3MZ_OK;
}

struct ActiveGuard {
  explicit ActiveGuard(p3mz_ctx* c) { g_active = c; }
  ~ActiveGuard() { g_active = nullptr; }
};

// The mesh step on positions `pos` (launch order: [pre] [cycles...] [post1]
// [post2], with the stage events between the launches).
p3mz_status mesh_step(p3mz_ctx* c, const double* pos, double* force, double* energy, hipStream_t s,
                      std::vector<uint64_t> post2_key, bool md, const MdArgs* m) {
  const uint64_t tm = c->timing;
  c->sub_events = false;
  c->ran_graphs = false;
  stage(c, 0, s);
  P3MZ_TRY(run_seq(c, c->g_pre, {(uint64_t)(uintptr_t)pos, tm}, s, [&](hipStream_t q) { return enq_pre(c, pos, q); }));
  P3MZ_TRY(run_solve(c, force, s));
  if (c->h_ctl->nan_flag) return on_nan(c);
  if (md)
    P3MZ_TRY(run_seq(c, c->g_md_post2, post2_key, s, [&](hipStream_t q) { return enq_md_post2(c, *m, q); }));
  else
    P3MZ_TRY(run_seq(c, c->g_post2, post2_key, s, [&](hipStream_t q) { return enq_post2(c, pos, force, energy, q); }));
  stage(c, 4, s);
  return P3MZ_OK;
}

p3mz_status compute_step(p3mz_ctx* c, const double* pos, double* force, double* energy, hipStream_t s) {
  ActiveGuard guard(c);
  P3MZ_TRY(mesh_step(c, pos, force, energy, s,
                     {(uint64_t)(uintptr_t)pos, (uint64_t)(uintptr_t)force, (uint64_t)(uintptr_t)energy}, false,
                     nullptr));
  P3MZ_TRY(finish(c, s));
  if (c->st.status) {
    g_last_error = "V-cycle cap reached before the tolerance";
    return P3MZ_WARN_NOT_CONVERGED;
  }
  return P3MZ_OK;
}

// ---------------------------------------------------------------------------
// Batched replicas.  A batch owns one ordinary context per system.  Each
// part of the step (kick, pre, one cycle, post1, post2) is enqueued once per
// system with a Recorder installed; the recorded launches of all systems are
// merged by sequence key into one k_many launch per key (blockIdx.y = system),
// so every launch of the batched step covers every system that has that
// launch, and each system's own order is kept.  Systems that converge earlier
// return from the remaining cycle kernels through their own control block.
// ---------------------------------------------------------------------------
struct BatchLaunch {
  ManyFn many;
  size_t off;   // byte offset of the packed arguments in the set's device block
  int count, gx;
  size_t lds;
};

enum { BQ_KICK = 0, BQ_PRE, BQ_CYCLE, BQ_POST1, BQ_POST2, BQ_EXTRA, BQ_COUNT };

struct BatchSet {
  std::vector<uint64_t> key;           // caller pointers/values the launches were recorded with
  std::vector<BatchLaunch> q[BQ_COUNT];
  void* d_args = nullptr;
  size_t cap = 0;
  GraphSlot g[BQ_COUNT];
  void drop() {
    for (GraphSlot& x : g) x.reset();
    key.clear();
  }
};

__global__ void k_batch_head(const Ctl* const* __restrict__ ctls, int n, int* __restrict__ out) {
  __shared__ int all_done, any_nan, cmax;
  if (threadIdx.x == 0) {
    all_done = 1;
    any_nan = 0;
    cmax = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const Ctl* c = ctls[i];
    if (!c->done) atomicAnd(&all_done, 0);
    if (c->nan_flag) atomicOr(&any_nan, 1);
    atomicMax(&cmax, c->cycles);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = all_done;
    out[1] = any_nan;
    out[2] = cmax;
  }
}

// Copies every system's control block into one array (one workgroup each).
__global__ void k_batch_collect(const Ctl* const* __restrict__ ctls, Ctl* __restrict__ dst) {
  const int* src = reinterpret_cast<const int*>(ctls[blockIdx.x]);
  int* d = reinterpret_cast<int*>(dst + blockIdx.x);
  for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int)); i += blockDim.x) d[i] = src[i];
}

__global__ void k_batch_md_reset(Ctl* const* __restrict__ ctls, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ctls[i]->md_step = 0;
}

}  // namespace

struct p3mz_batch {
  std::vector<p3mz_ctx*> sys;
  std::vector<int64_t> off;        // first atom of each system in the packed arrays
  int64_t n_total = 0;
  bool fp64 = false;
  Ctl** d_ctls = nullptr;          // device array of the systems' control blocks
  Ctl* d_ctl_all = nullptr;        // collected control blocks
  Ctl* h_ctl_all = nullptr;        // pinned
  int* d_head = nullptr;
  int* h_head = nullptr;           // pinned {all done, any nan, max cycles}
  BatchSet compute, md;
  bool use_graphs = true;
  bool md_have_force = false;
  std::vector<uint64_t> md_force_key;   // buffers and terms the systems' forces were computed with
  int last_cycles = 0;
  hipStream_t cap = nullptr;
  bool timing = false;
  hipEvent_t ev[3] = {};
  double ms_mesh = 0.0, ms_sr = 0.0;
  int ran_graphs = 0;
  int64_t steps = 0;
  ~p3mz_batch() {
    compute.drop();
    md.drop();
    for (BatchSet* b : {&compute, &md})
      if (b->d_args) (void)hipFree(b->d_args);
    if (d_ctls) (void)hipFree(d_ctls);
    if (d_ctl_all) (void)hipFree(d_ctl_all);
    if (d_head) (void)hipFree(d_head);
    if (h_ctl_all) (void)hipHostFree(h_ctl_all);
    if (h_head) (void)hipHostFree(h_head);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    for (p3mz_ctx* c : sys) delete c;
  }
};

namespace {

// Record part `part` of every system with enq(system index) and merge the
// launches by key into set->q[part]; packed arguments are appended to `args`.
template <typename F>
p3mz_status batch_record(p3mz_batch* b, BatchSet* set, int part, std::vector<unsigned char>* args, F enq) {
  const int R = (int)b->sys.size();
  std::vector<std::vector<LaunchRec>> recs(R);
  for (int r = 0; r < R; r++) {
    Recorder rec;
    g_recorder = &rec;
    p3mz_status st = enq(r);
    g_recorder = nullptr;
    if (st != P3MZ_OK) return st;
    for (size_t i = 1; i < rec.recs.size(); i++)
      if (rec.recs[i].key <= rec.recs[i - 1].key) return fail(P3MZ_ERR_STATE, "internal: launch keys out of order");
    recs[r] = std::move(rec.recs);
  }
  std::vector<size_t> pos(R, 0);
  std::vector<BatchLaunch>& out = set->q[part];
  out.clear();
  for (;;) {
    uint32_t k = UINT32_MAX;
    for (int r = 0; r < R; r++)
      if (pos[r] < recs[r].size()) k = std::min(k, recs[r][pos[r]].key);
    if (k == UINT32_MAX) break;
    BatchLaunch L{nullptr, 0, 0, 0, 0};
    size_t elem = 0;
    args->resize((args->size() + 255) & ~(size_t)255);
    L.off = args->size();
    for (int r = 0; r < R; r++) {
      if (pos[r] >= recs[r].size() || recs[r][pos[r]].key != k) continue;
      const LaunchRec& x = recs[r][pos[r]++];
      if (!L.many) {
        L.many = x.many;
        elem = x.args.size();
      } else if (L.many != x.many || elem != x.args.size()) {
        return fail(P3MZ_ERR_STATE, "systems of one batch need the same precision and sweep structure");
      }
      const size_t at = args->size();
      args->insert(args->end(), x.args.begin(), x.args.end());
      const int first = L.gx;   // this system's workgroups follow the previous ones
      memcpy(args->data() + at + x.off_field, &first, sizeof first);
      L.count++;
      L.gx += x.grid;
      L.lds = std::max(L.lds, x.lds);
    }
    // round the grid up to a multiple of 8 so the XCD renumbering applies
    if (L.gx >= 8) L.gx = (L.gx + 7) & ~7;
    out.push_back(L);
  }
  return P3MZ_OK;
}

p3mz_status batch_upload(BatchSet* set, const std::vector<unsigned char>& args) {
  // launches of the previous recording may still read the old arguments
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  if (args.size() > set->cap) {
    if (set->d_args) P3MZ_HIP_TRY(hipFree(set->d_args));
    set->d_args = nullptr;
    set->cap = 0;
    P3MZ_HIP_TRY(hipMalloc(&set->d_args, args.size()));
    set->cap = args.size();
  }
  if (!args.empty()) P3MZ_HIP_TRY(hipMemcpy(set->d_args, args.data(), args.size(), hipMemcpyHostToDevice));
  return P3MZ_OK;
}

p3mz_status batch_run_part(p3mz_batch* b, BatchSet* set, int part, hipStream_t s) {
  auto body = [&](hipStream_t q) -> p3mz_status {
    for (const BatchLaunch& L : set->q[part])
      P3MZ_HIP_TRY(L.many((const char*)set->d_args + L.off, L.count, L.gx, L.lds, q));
    return P3MZ_OK;
  };
  if (set->q[part].empty()) return P3MZ_OK;
  if (!b->use_graphs) return body(s);
  GraphSlot& slot = set->g[part];
  if (!slot.exec) {
    slot.reset();
    P3MZ_HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    p3mz_status st = body(b->cap);
    hipError_t e = hipStreamEndCapture(b->cap, &slot.graph);
    if (st != P3MZ_OK || e != hipSuccess || hipGraphInstantiate(&slot.exec, slot.graph, nullptr, nullptr, 0) != hipSuccess) {
      slot.reset();
      (void)hipGetLastError();
      b->use_graphs = false;
      return body(s);
    }
  }
  P3MZ_HIP_TRY(hipGraphLaunch(slot.exec, s));
  b->ran_graphs = 1;
  return P3MZ_OK;
}

p3mz_status batch_read_head(p3mz_batch* b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_head, dim3(1), dim3(256), 0, s, (const Ctl* const*)b->d_ctls, (int)b->sys.size(),
                     b->d_head);
  P3MZ_HIP_TRY(hipGetLastError());
  P3MZ_HIP_TRY(hipMemcpyAsync(b->h_head, b->d_head, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  P3MZ_HIP_TRY(hipStreamSynchronize(s));
  return P3MZ_OK;
}

// Statistics of every system after a batched step, from one collected copy
// of all control blocks (same fields as a single context's finish()).
p3mz_status batch_finish(p3mz_batch* b, hipStream_t s) {
  const int R = (int)b->sys.size();
  hipLaunchKernelGGL(k_batch_collect, dim3(R), dim3(64), 0, s, (const Ctl* const*)b->d_ctls, b->d_ctl_all);
  P3MZ_HIP_TRY(hipGetLastError());
  P3MZ_HIP_TRY(hipMemcpyAsync(b->h_ctl_all, b->d_ctl_all, R * sizeof(Ctl), hipMemcpyDeviceToHost, s));
  P3MZ_HIP_TRY(hipStreamSynchronize(s));
  int cmax = 0;
  for (int r = 0; r < R; r++) {
    p3mz_ctx* c = b->sys[r];
    const Ctl& h = b->h_ctl_all[r];
    const int was_cold = c->mirror.cold, m_eff = c->mirror.m_eff;
    c->mirror = h;
    *c->h_ctl = h;
    c->last_cycles = h.cycles;
    cmax = std::max(cmax, h.cycles);
    p3mz_stats& st = c->st;
    st.status = h.status ? P3MZ_WARN_NOT_CONVERGED : P3MZ_OK;
    st.cycles = h.cycles;
    st.cold = was_cold;
    st.m_eff = m_eff;
    st.nu_pre = c->nu1;
    st.nu_post = c->nu2;
    st.K = c->pl.K;
    st.levels = c->pl.levels;
    st.nu_smooth = c->pl.nu_s;
    st.thresh = h.thresh;
    st.norm_qs = h.norm_qs;
    for (int i = 0; i <= P3MZ_MAX_CYCLES; i++) st.res_hist[i] = i <= h.cycles ? h.res_hist[i] : 0.0;
    st.e_sr = h.e_sr;
    st.e_lr = h.e_lr;
    st.e_self = c->e_self;
    st.e_total = h.e_sr + h.e_lr + c->e_self;
    st.steps = h.steps;
    st.graphs = b->ran_graphs;
    for (int k = 0; k < 3; k++) st.net_force[k] = h.net_force[k];
    st.ms_mesh = st.ms_short_range = st.ms_spread = st.ms_solve = st.ms_gather = -1.0;
  }
  b->last_cycles = cmax;
  if (b->timing) {
    float ms = 0.f;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
    b->ms_mesh = ms;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, b->ev[1], b->ev[2]));
    b->ms_sr = ms;
  }
  return P3MZ_OK;
}

// One batched mesh step with the launches of `set` (kick and extra parts run
// when `kick` / `extra` are set).  Returns NAN when a system saw a non-finite
// position (that system's history is dropped, as for a single context).
p3mz_status batch_step(p3mz_batch* b, BatchSet* set, hipStream_t s, bool kick, bool extra, bool* not_converged) {
  b->ran_graphs = 0;
  if (kick) P3MZ_TRY(batch_run_part(b, set, BQ_KICK, s));
  if (b->timing) P3MZ_HIP_TRY(hipEventRecord(b->ev[0], s));
  P3MZ_TRY(batch_run_part(b, set, BQ_PRE, s));
  int max_c = 0;
  for (p3mz_ctx* c : b->sys) max_c = std::max(max_c, c->P.max_cycles);
  int issued = 0, batch = std::max(1, b->last_cycles);
  for (;;) {
    for (int k = 0; k < batch && issued < max_c; k++, issued++) P3MZ_TRY(batch_run_part(b, set, BQ_CYCLE, s));
    P3MZ_TRY(batch_read_head(b, s));
    if (b->h_head[0] || b->h_head[1] || issued >= max_c) break;
    batch = 1;
  }
  if (b->h_head[1]) {
    P3MZ_TRY(batch_finish(b, s));
    for (p3mz_ctx* c : b->sys)
      if (c->mirror.nan_flag) (void)on_nan(c);
    b->md_have_force = false;
    b->last_cycles = 0;
    return fail(P3MZ_ERR_NAN, "non-finite position in a batched system");
  }
  P3MZ_TRY(batch_run_part(b, set, BQ_POST1, s));
  if (b->timing) P3MZ_HIP_TRY(hipEventRecord(b->ev[1], s));
  P3MZ_TRY(batch_run_part(b, set, BQ_POST2, s));
  if (extra) P3MZ_TRY(batch_run_part(b, set, BQ_EXTRA, s));
  if (b->timing) P3MZ_HIP_TRY(hipEventRecord(b->ev[2], s));
  P3MZ_TRY(batch_finish(b, s));
  bool nc = false;
  for (p3mz_ctx* c : b->sys) nc |= c->st.status != P3MZ_OK;
  *not_converged = nc;
  b->steps++;
  return P3MZ_OK;
}

MdArgs md_args_for(const p3mz_mdterms* t, double dt) {
  MdArgs m{};
  m.dt = dt;
  m.f2a = t->force_to_acc;
  m.mv2e = t->mv2_to_energy;
  m.model = t->model;
  if (t->model == 1) {
    m.p[0] = t->bm_a;
    m.p[1] = t->bm_rho;
  } else if (t->model == 2) {
    m.p[0] = t->lj_eps; m.p[1] = t->lj_sigma; m.p[2] = t->k_bond; m.p[3] = t->r0;
    m.p[4] = t->k_angle; m.p[5] = t->theta0;
  }
  return m;
}

std::vector<uint64_t> md_key(const MdArgs& m) {
  std::vector<uint64_t> k = {(uint64_t)m.model, bits(m.dt), bits(m.f2a), bits(m.mv2e)};
  for (double v : m.p) k.push_back(bits(v));
  return k;
}

// (Re)record the compute set for caller buffers pos/force/energy (packed;
// force and energy NULL: each system's internal MD buffers).  With `init`
// (forces before the first MD step) the non-electrostatic terms are added.
p3mz_status batch_prepare_compute(p3mz_batch* b, const double* pos, double* force, double* energy,
                                  const MdArgs* init) {
  std::vector<uint64_t> key = {(uint64_t)(uintptr_t)pos, (uint64_t)(uintptr_t)force, (uint64_t)(uintptr_t)energy,
                               (uint64_t)(init != nullptr)};
  if (init) {
    const std::vector<uint64_t> k2 = md_key(*init);
    key.insert(key.end(), k2.begin(), k2.end());
  }
  if (b->compute.key == key) return P3MZ_OK;
  b->compute.drop();
  std::vector<unsigned char> args;
  auto F = [&](int r) { return force ? force + 3 * b->off[r] : b->sys[r]->d_md_force; };
  auto E = [&](int r) { return energy ? energy + 4 * r : b->sys[r]->d_energy; };
  auto X = [&](int r) { return pos + 3 * b->off[r]; };
  P3MZ_TRY(batch_record(b, &b->compute, BQ_PRE, &args, [&](int r) { return enq_pre(b->sys[r], X(r), nullptr); }));
  P3MZ_TRY(batch_record(b, &b->compute, BQ_CYCLE, &args, [&](int r) { return enq_cycle(b->sys[r], nullptr); }));
  P3MZ_TRY(batch_record(b, &b->compute, BQ_POST1, &args,
                        [&](int r) { return enq_post1(b->sys[r], F(r), nullptr); }));
  P3MZ_TRY(batch_record(b, &b->compute, BQ_POST2, &args,
                        [&](int r) { return enq_post2(b->sys[r], X(r), F(r), E(r), nullptr); }));
  b->compute.q[BQ_KICK].clear();
  b->compute.q[BQ_EXTRA].clear();
  if (init) {
    P3MZ_TRY(batch_record(b, &b->compute, BQ_EXTRA, &args, [&](int r) -> p3mz_status {
      p3mz_ctx* c = b->sys[r];
      rec_key(6100);
      P3MZ_HIP_TRY(launch_nonelec((int)c->n_atoms, X(r), c->P.box, c->P.r_cut, init->model, init->p[0], init->p[1],
                                  init->p[2], init->p[3], init->p[4], init->p[5], c->nc, c->d_cstart, c->d_cperm, c->d_spos,
                                  c->d_md_force, c->d_partial, c->d_e_other, nullptr));
      return P3MZ_OK;
    }));
  }
  P3MZ_TRY(batch_upload(&b->compute, args));
  b->compute.key = key;
  return P3MZ_OK;
}

// (Re)record the MD set: kick + drift, mesh step, pairs, non-electrostatic
// terms, closing kick and the per-system logs ([system][step] rows).
p3mz_status batch_prepare_md(p3mz_batch* b, double* pos, double* vel, const double* mass, const MdArgs& m0,
                             double* elog, int32_t* clog, int n_steps) {
  std::vector<uint64_t> key = {(uint64_t)(uintptr_t)pos, (uint64_t)(uintptr_t)vel, (uint64_t)(uintptr_t)mass,
                               (uint64_t)(uintptr_t)elog, (uint64_t)(uintptr_t)clog, (uint64_t)n_steps};
  const std::vector<uint64_t> k2 = md_key(m0);
  key.insert(key.end(), k2.begin(), k2.end());
  if (b->md.key == key) return P3MZ_OK;
  b->md.drop();
  std::vector<unsigned char> args;
  auto M = [&](int r) {
    MdArgs m = m0;
    m.pos = pos + 3 * b->off[r];
    m.vel = vel + 3 * b->off[r];
    m.mass = mass + b->off[r];
    m.elog = elog ? elog + (size_t)6 * n_steps * r : nullptr;
    m.clog = clog ? clog + (size_t)n_steps * r : nullptr;
    return m;
  };
  P3MZ_TRY(batch_record(b, &b->md, BQ_KICK, &args, [&](int r) -> p3mz_status {
    p3mz_ctx* c = b->sys[r];
    const MdArgs m = M(r);
    rec_key(90);
    P3MZ_HIP_TRY(launch_kick_drift((int)c->n_atoms, m.pos, m.vel, c->d_md_force, m.mass, m.dt, m.f2a, 1, nullptr));
    return P3MZ_OK;
  }));
  P3MZ_TRY(batch_record(b, &b->md, BQ_PRE, &args, [&](int r) { return enq_pre(b->sys[r], M(r).pos, nullptr); }));
  P3MZ_TRY(batch_record(b, &b->md, BQ_CYCLE, &args, [&](int r) { return enq_cycle(b->sys[r], nullptr); }));
  P3MZ_TRY(batch_record(b, &b->md, BQ_POST1, &args,
                        [&](int r) { return enq_post1(b->sys[r], b->sys[r]->d_md_force, nullptr); }));
  P3MZ_TRY(batch_record(b, &b->md, BQ_POST2, &args, [&](int r) { return enq_md_post2(b->sys[r], M(r), nullptr); }));
  b->md.q[BQ_EXTRA].clear();
  P3MZ_TRY(batch_upload(&b->md, args));
  b->md.key = key;
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
  ctx->md_have_force = false;
  return compute_step(ctx, pos_dev, force_dev, energy_dev, (hipStream_t)stream);
}

p3mz_status p3mz_get_mesh(p3mz_ctx* ctx, int32_t which, double* out_dev, void* stream) {
  if (!ctx || !out_dev) return fail(P3MZ_ERR_INVALID_ARG, "ctx or out_dev is NULL");
  hipStream_t s = (hipStream_t)stream;
  const size_t n3 = (size_t)ctx->n3;
  const Ctl& m = ctx->mirror;
  switch (which) {
    case 0: P3MZ_HIP_TRY(launch_widen(!ctx->src32, (int64_t)n3, ctx->d_q, out_dev, s)); break;
    case 1: P3MZ_HIP_TRY(launch_widen(!ctx->src32, (int64_t)n3, ctx->d_qs, out_dev, s)); break;
    case 2: P3MZ_HIP_TRY(launch_sub_scalar(n3, ctx->d_sigma, out_dev, &ctx->d_ctl->mean_sigma, s)); break;
    case 3: {
      // the final multiplier after the zero-mean projection is the newest
      // stored one after a warm step; a cold solve stores none
      if (ctx->st.cold) return fail(P3MZ_ERR_STATE, "multiplier of a cold solve is not kept");
      const int slot = m.yh0;
      P3MZ_HIP_TRY(hipMemcpyAsync(out_dev, ctx->d_yh[slot], n3 * 8, hipMemcpyDeviceToDevice, s));
      break;
    }
    case 4: P3MZ_HIP_TRY(hipMemcpyAsync(out_dev, ctx->d_phi[m.k_idx], n3 * 8, hipMemcpyDeviceToDevice, s)); break;
    case 5: P3MZ_HIP_TRY(hipMemcpyAsync(out_dev, ctx->d_phi[1 - m.k_idx], n3 * 8, hipMemcpyDeviceToDevice, s)); break;
    default: return fail(P3MZ_ERR_INVALID_ARG, "unknown mesh id");
  }
  return P3MZ_OK;
}

p3mz_status p3mz_get_potential(p3mz_ctx* ctx, double* phi_dev, void* stream) {
  return p3mz_get_mesh(ctx, 4, phi_dev, stream);
}

p3mz_status p3mz_vcycle(p3mz_ctx* ctx, const double* r_dev, double* e_dev, void* stream) {
  if (!ctx || !r_dev || !e_dev) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const LevelBufs& f = ctx->lv[0];
  P3MZ_HIP_TRY(launch_set_ctl_open(ctx->d_ctl, s));
  P3MZ_HIP_TRY(launch_nat_to_cs(ctx->fp64, ctx->pl.n, r_dev, f.r0, f.r1, s));
  P3MZ_HIP_TRY(launch_vcycle(ctx->fp64, ctx->lv, ctx->pl.levels, ctx->pl.tail, ctx->nu1, ctx->nu2, ctx->d_green,
                             ctx->d_ctl, s));
  P3MZ_HIP_TRY(launch_cs_to_nat(ctx->fp64, ctx->pl.n, cycle_e0(f, ctx->fp64, ctx->nu2), cycle_e1(f, ctx->fp64, ctx->nu2),
                                e_dev, s));
  return P3MZ_OK;
}

p3mz_status p3mz_get_stats(const p3mz_ctx* ctx, p3mz_stats* out) {
  if (!ctx || !out) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  *out = ctx->st;
  return P3MZ_OK;
}

p3mz_status p3mz_reset_history(p3mz_ctx* ctx) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  P3MZ_HIP_TRY(hipMemcpy(&ctx->mirror, ctx->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  ctx->mirror.cold = 1;
  ctx->mirror.n_yh = 0;
  ctx->mirror.m_eff = 0;
  P3MZ_HIP_TRY(hipMemcpy(ctx->d_ctl, &ctx->mirror, sizeof(Ctl), hipMemcpyHostToDevice));
  ctx->last_cycles = 0;
  ctx->md_have_force = false;
  return P3MZ_OK;
}

// blob: magic, n, precision, cold, n_yh, steps, last_cycles, then
// phi^k, phi^{k-1}, y^k, y^{k-1}, y^{k-2} (FP64, natural layout).
static const int64_t kMagic = 0x50334d5a53543032LL;   // "P3MZST02"

p3mz_status p3mz_save_state(const p3mz_ctx* ctx, void* host_buf, size_t* bytes) {
  if (!ctx || !bytes) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  const size_t n3 = (size_t)ctx->n3;
  const size_t need = 7 * sizeof(int64_t) + 5 * n3 * sizeof(double);
  if (!host_buf) {
    *bytes = need;
    return P3MZ_OK;
  }
  if (*bytes < need) return fail(P3MZ_ERR_INVALID_ARG, "buffer too small");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  Ctl m;
  P3MZ_HIP_TRY(hipMemcpy(&m, ctx->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  int64_t hdr[7] = {kMagic, ctx->pl.n, ctx->P.precision, m.cold, m.n_yh, m.steps, ctx->last_cycles};
  char* b = (char*)host_buf;
  memcpy(b, hdr, sizeof hdr);
  b += sizeof hdr;
  const double* arr[5] = {ctx->d_phi[m.k_idx], ctx->d_phi[1 - m.k_idx], ctx->d_yh[m.yh0], ctx->d_yh[m.yh1],
                          ctx->d_yh[m.yh2]};
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
  if (hdr[0] != kMagic || hdr[1] != ctx->pl.n || hdr[2] != ctx->P.precision || hdr[4] < 0 || hdr[4] > 3 ||
      hdr[3] < 0 || hdr[3] > 1)
    return fail(P3MZ_ERR_STATE, "state blob does not match this context");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  double* arr[5] = {ctx->d_phi[0], ctx->d_phi[1], ctx->d_yh[0], ctx->d_yh[1], ctx->d_yh[2]};
  for (int i = 0; i < 5; i++) {
    P3MZ_HIP_TRY(hipMemcpy(arr[i], b, n3 * 8, hipMemcpyHostToDevice));
    b += n3 * 8;
  }
  P3MZ_HIP_TRY(hipMemcpy(&ctx->mirror, ctx->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  Ctl& m = ctx->mirror;
  m.cold = (int)hdr[3];
  m.n_yh = (int)hdr[4];
  m.steps = hdr[5];
  m.k_idx = 0;
  m.yh0 = 0;
  m.yh1 = 1;
  m.yh2 = 2;
  m.m_eff = m.cold ? 0 : std::min(ctx->P.predictor, m.n_yh);
  m.nan_flag = 0;
  P3MZ_HIP_TRY(hipMemcpy(ctx->d_ctl, &m, sizeof(Ctl), hipMemcpyHostToDevice));
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
  ActiveGuard guard(ctx);
  MdArgs m{};
  m.pos = pos_dev;
  m.vel = vel_dev;
  m.mass = mass_dev;
  m.elog = energy_log_dev;
  m.clog = cycles_log_dev;
  m.dt = dt;
  m.f2a = terms->force_to_acc;
  m.mv2e = terms->mv2_to_energy;
  m.model = terms->model;
  m.th = Thermostat{0, 1.0, 0.0, 0.0, 1.0, 0u, 0u, nullptr};
  if (ctx->th_gamma > 0.0) {
    const double a = exp(-0.5 * ctx->th_gamma * dt);
    m.th = Thermostat{1, a, sqrt(1.0 - a * a), ctx->th_kt, m.mv2e, (unsigned)ctx->th_seed,
                      (unsigned)(ctx->th_seed >> 32), ctx->d_ctl};
  }
  if (terms->model == 1) {
    m.p[0] = terms->bm_a;
    m.p[1] = terms->bm_rho;
  } else if (terms->model == 2) {
    m.p[0] = terms->lj_eps; m.p[1] = terms->lj_sigma; m.p[2] = terms->k_bond; m.p[3] = terms->r0;
    m.p[4] = terms->k_angle; m.p[5] = terms->theta0;
  }
  std::vector<uint64_t> key_post2 = {(uint64_t)(uintptr_t)pos_dev, (uint64_t)(uintptr_t)vel_dev,
                                     (uint64_t)(uintptr_t)mass_dev, bits(dt), bits(m.f2a),
                                     (uint64_t)(uintptr_t)energy_log_dev, (uint64_t)(uintptr_t)cycles_log_dev,
                                     (uint64_t)m.model, bits(m.mv2e)};
  for (double v : m.p) key_post2.push_back(bits(v));
  for (double v : {m.th.a, m.th.b, m.th.kt}) key_post2.push_back(bits(v));
  key_post2.push_back(ctx->th_seed);
  key_post2.push_back((uint64_t)m.th.on);
  P3MZ_HIP_TRY(hipMemsetAsync(&ctx->d_ctl->md_step, 0, sizeof(int), s));   // eager, never captured
  // the stored forces continue a trajectory only for the same buffers and terms
  std::vector<uint64_t> force_key = {(uint64_t)(uintptr_t)pos_dev, (uint64_t)(uintptr_t)vel_dev,
                                     (uint64_t)(uintptr_t)mass_dev, (uint64_t)m.model};
  for (double v : m.p) force_key.push_back(bits(v));
  if (ctx->md_have_force && ctx->md_force_key != force_key) ctx->md_have_force = false;
  if (!ctx->md_have_force) {
    // forces at the initial positions (a cold solve on first use); no log row
    P3MZ_TRY(mesh_step(ctx, pos_dev, ctx->d_md_force, ctx->d_energy, s,
                       {(uint64_t)(uintptr_t)pos_dev, (uint64_t)(uintptr_t)ctx->d_md_force,
                        (uint64_t)(uintptr_t)ctx->d_energy},
                       false, nullptr));
    P3MZ_HIP_TRY(launch_nonelec((int)ctx->n_atoms, pos_dev, ctx->P.box, ctx->P.r_cut, m.model, m.p[0], m.p[1], m.p[2],
                                m.p[3], m.p[4], m.p[5], ctx->nc, ctx->d_cstart, ctx->d_cperm, ctx->d_spos, ctx->d_md_force,
                                ctx->d_partial, ctx->d_e_other, s, ctx->d_nbr, ctx->d_nlist, ctx->nbr_cap));
    P3MZ_TRY(finish(ctx, s));
    ctx->md_have_force = true;
    ctx->md_force_key = force_key;
  }
  p3mz_status worst = P3MZ_OK;
  for (int step = 0; step < n_steps; step++) {
    P3MZ_HIP_TRY(launch_kick_drift((int)ctx->n_atoms, pos_dev, vel_dev, ctx->d_md_force, mass_dev, dt, m.f2a, 1, s,
                                   &m.th));
    P3MZ_TRY(mesh_step(ctx, pos_dev, ctx->d_md_force, ctx->d_energy, s, key_post2, true, &m));
    if (ctx->h_ctl->status) worst = P3MZ_WARN_NOT_CONVERGED;
    ctx->last_cycles = ctx->h_ctl->cycles;
  }
  P3MZ_TRY(finish(ctx, s));
  return worst;
}

p3mz_status p3mz_set_timing(p3mz_ctx* ctx, int32_t on) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (on && !ctx->stage_ev[0])
    for (hipEvent_t& e : ctx->stage_ev) P3MZ_HIP_TRY(hipEventCreate(&e));
  ctx->timing = on != 0;
  ctx->st.ms_mesh = ctx->st.ms_short_range = 0.0;
  ctx->st.ms_spread = ctx->st.ms_solve = ctx->st.ms_gather = -1.0;
  return P3MZ_OK;
}

p3mz_status p3mz_set_graphs(p3mz_ctx* ctx, int32_t on) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  ctx->drop_graphs();
  ctx->use_graphs = on != 0;
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
  ctx->kt_hist_ms.clear();
  ctx->kt_hist_bytes.clear();
  return P3MZ_OK;
}

p3mz_status p3mz_get_kernel_launches(const p3mz_ctx* ctx, int32_t max, float* ms_host, double* bytes_host,
                                     int32_t* count) {
  if (!ctx || !ms_host || !bytes_host || !count || max < 0) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  const int32_t n = (int32_t)std::min<size_t>((size_t)max, ctx->kt_hist_ms.size());
  for (int32_t i = 0; i < n; i++) {
    ms_host[i] = ctx->kt_hist_ms[(size_t)i];
    bytes_host[i] = ctx->kt_hist_bytes[(size_t)i];
  }
  *count = n;
  return P3MZ_OK;
}

p3mz_status p3mz_get_kernel_timer(const p3mz_ctx* ctx, double* total_ms, int64_t* launches, double* total_bytes) {
  if (!ctx || !total_ms || !launches || !total_bytes) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  *total_ms = ctx->kt_total_ms;
  *launches = ctx->kt_launches;
  *total_bytes = ctx->kt_total_bytes;
  return P3MZ_OK;
}

p3mz_status p3mz_kernel_bench(p3mz_ctx* ctx, int32_t kernel_id, int32_t reps, void* stream, double* avg_ms,
                              double* bytes_per_launch) {
  if (!ctx || !avg_ms || !bytes_per_launch || reps < 1) return fail(P3MZ_ERR_INVALID_ARG, "bad kernel_bench arguments");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  P3MZ_HIP_TRY(hipEventCreate(&e0));
  P3MZ_HIP_TRY(hipEventCreate(&e1));
  double bytes = 0.0;
  p3mz_status st = P3MZ_OK;
  P3MZ_HIP_TRY(launch_set_ctl_open(ctx->d_ctl, s));
  P3MZ_HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps && st == P3MZ_OK; r++) {
    hipError_t e;
    const double N3 = (double)ctx->n3, na = (double)ctx->n_atoms, ts = (double)ctx->tsz;
    const int p = ctx->pl.p, n = ctx->pl.n;
    const LevelBufs& f = ctx->lv[0];
    if (kernel_id == KT_SMOOTH) {
      e = launch_smooth(!ctx->src32, ctx->pl.n, 0, ctx->smooth_tile, ctx->ntaps, ctx->half, ctx->d_taps, ctx->d_q,
                        ctx->d_tmp, s);
      bytes = (ctx->src32 ? 8.0 : 16.0) * N3;
    } else if (kernel_id == KT_OUTER) {
      // the cycle form without its finalize pass; both multiplier buffers
      // are scratch between steps (the multiplier is kept in the history slots)
      e = launch_outer(ctx->fp64, n, 0, ctx->P.max_cycles, ctx->d_sigma, ctx->d_y[0], ctx->d_y[1],
                       cycle_e0(f, ctx->fp64, ctx->nu2), cycle_e1(f, ctx->fp64, ctx->nu2), f.r0,
                       f.r1, ctx->d_partial, ctx->d_ctl, s, false, nullptr, 0.0, 0, ctx->P.stencil);
      bytes = (24.0 + 2.0 * ts) * N3;
    } else if (kernel_id == KT_SIGMA) {
      e = launch_sigma(n, ctx->pl.h, ctx->src32, ctx->d_qs, ctx->d_phi[0], ctx->d_phi[1], ctx->d_yh[0], ctx->d_yh[1],
                       ctx->d_yh[2], ctx->d_sigma, ctx->d_y[0], ctx->P.tol, ctx->P.tol_mode, ctx->d_partial, ctx->d_ctl,
                       s, false, ctx->P.stencil);
      bytes = (ctx->src32 ? 60.0 : 64.0) * N3;
    } else if (kernel_id == KT_SPREAD) {
      e = launch_spread(!ctx->src32, n, p, kTile, ctx->ntx, ctx->P.box, ctx->d_start, ctx->d_cls, ctx->d_rb, ctx->d_rq,
                        ctx->d_tmp, s);
      bytes = (ctx->src32 ? 4.0 : 8.0) * N3 + 40.0 * na;
    } else if (kernel_id == KT_GATHER) {
      e = launch_gather(ctx->fp64, (int)ctx->n_atoms, n, p, kTile, ctx->ntx, ctx->pl.h, ctx->P.coulomb_k, ctx->d_start,
                        ctx->d_rb, ctx->d_rq, ctx->d_phi[0], ctx->d_phi[1], ctx->d_phi32, nullptr,
                        ctx->d_partial, ctx->d_ctl, s, false, ctx->P.stencil);
      bytes = N3 * (ctx->fp64 ? 8.0 : 4.0) + 64.0 * na;
    } else {
      e = launch_vcycle_kernel(ctx->fp64, kernel_id, ctx->lv, ctx->pl.levels, ctx->pl.tail, ctx->nu1, ctx->nu2,
                               ctx->d_green, ctx->d_ctl, s, &bytes);
    }
    if (e != hipSuccess) st = fail(P3MZ_ERR_INVALID_ARG, "kernel not available for timing on this mesh");
  }
  P3MZ_HIP_TRY(hipEventRecord(e1, s));
  P3MZ_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  P3MZ_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the control block now says "open"; the next compute resets it anyway
  *avg_ms = ms / reps;
  *bytes_per_launch = bytes;
  return st;
}

p3mz_status p3mz_set_schedule(p3mz_ctx* ctx, int32_t nu_pre, int32_t nu_post, int32_t smooth_tile) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (nu_pre < 0 || nu_post < 0 || nu_pre > 16 || nu_post > 16 || nu_pre + nu_post < 1)
    return fail(P3MZ_ERR_INVALID_ARG, "sweep counts must be in 0..16 with nu_pre + nu_post >= 1");
  if (!smooth_tile_ok(smooth_tile, ctx->pl.n, ctx->ntaps)) return fail(P3MZ_ERR_INVALID_ARG, "smoothing tile not valid on this mesh");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  ctx->drop_graphs();
  ctx->nu1 = nu_pre;
  ctx->nu2 = nu_post;
  ctx->smooth_tile = smooth_tile;
  return P3MZ_OK;
}

p3mz_status p3mz_set_fused_levels(p3mz_ctx* ctx, int32_t max_edge) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (max_edge < 0) return fail(P3MZ_ERR_INVALID_ARG, "max_edge must be >= 0");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  ctx->drop_graphs();
  for (int l = 0; l < ctx->pl.levels; l++) {
    LevelBufs& b = ctx->lv[l];
    b.fty = b.ftz = (b.d0 && b.n <= max_edge) ? fused_tile(b.n) : 0;
  }
  return P3MZ_OK;
}

p3mz_status p3mz_set_neighbor_list(p3mz_ctx* ctx, double skin, int32_t capacity) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (!(skin >= 0.0) || !(skin <= ctx->P.r_cut) || capacity < 0)
    return fail(P3MZ_ERR_INVALID_ARG, "skin must be in [0, r_cut] and capacity >= 0");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  return nbr_configure(ctx, skin, capacity);
}

p3mz_status p3mz_set_thermostat(p3mz_ctx* ctx, double gamma, double kt, uint64_t seed) {
  if (!ctx) return fail(P3MZ_ERR_INVALID_ARG, "ctx is NULL");
  if (!(gamma >= 0.0) || !(kt >= 0.0) || !isfinite(gamma) || !isfinite(kt))
    return fail(P3MZ_ERR_INVALID_ARG, "gamma and kT must be finite and >= 0");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  ctx->th_gamma = gamma;
  ctx->th_kt = kt;
  ctx->th_seed = seed;
  const long long zero = 0;
  P3MZ_HIP_TRY(hipMemcpy(&ctx->d_ctl->therm_step, &zero, sizeof zero, hipMemcpyHostToDevice));
  return P3MZ_OK;
}

p3mz_status p3mz_get_neighbor_stats(const p3mz_ctx* ctx, int64_t* builds, int64_t* over_capacity,
                                    int32_t* capacity) {
  if (!ctx || !builds || !over_capacity || !capacity) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  *builds = ctx->mirror.nbr_builds;
  *over_capacity = ctx->mirror.nbr_over;
  *capacity = ctx->nbr_cap;
  return P3MZ_OK;
}

p3mz_status p3mz_autotune(p3mz_ctx* ctx, const double* frames_dev, int32_t n_frames, void* stream,
                          p3mz_tune_result* out) {
  if (!ctx || !frames_dev || n_frames < 1 || n_frames > 64 || !out)
    return fail(P3MZ_ERR_INVALID_ARG, "bad autotune arguments");
  hipStream_t s = (hipStream_t)stream;
  memset(out, 0, sizeof *out);
  const int n = ctx->pl.n;
  // 1. smoothing launch shape: the three axis passes back to back, best of 3
  hipEvent_t e0, e1;
  P3MZ_HIP_TRY(hipEventCreate(&e0));
  P3MZ_HIP_TRY(hipEventCreate(&e1));
  int best_tile = ctx->smooth_tile;
  double best_tile_ms = 1e300;
  for (int t = 0; t < smooth_tile_count(); t++) {
    if (!smooth_tile_ok(t, n, ctx->ntaps)) continue;
    double ms_min = 1e300;
    for (int rep = 0; rep < 4; rep++) {
      P3MZ_HIP_TRY(hipEventRecord(e0, s));
      double* src[3] = {ctx->d_q, ctx->d_tmp, ctx->d_qs};
      double* dst[3] = {ctx->d_tmp, ctx->d_qs, ctx->d_tmp};
      for (int axis = 0; axis < 3; axis++)
        P3MZ_HIP_TRY(launch_smooth(!ctx->src32, n, axis, t, ctx->ntaps, ctx->half, ctx->d_taps, src[axis], dst[axis],
                                   s));
      P3MZ_HIP_TRY(hipEventRecord(e1, s));
      P3MZ_HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      P3MZ_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) ms_min = std::min(ms_min, (double)ms);   // the first run warms up
    }
    if (ms_min < best_tile_ms) {
      best_tile_ms = ms_min;
      best_tile = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  out->smooth_tile = best_tile;
  out->ms_smooth = best_tile_ms;
  // 2. sweep schedule by time to tolerance over the caller's frames, each
  //    candidate starting from the same saved history
  size_t bytes = 0;
  P3MZ_TRY(p3mz_save_state(ctx, nullptr, &bytes));
  std::vector<char> blob(bytes);
  P3MZ_TRY(p3mz_save_state(ctx, blob.data(), &bytes));
  const int cand[][2] = {{2, 2}, {1, 1}, {1, 2}, {2, 1}, {0, 2}, {2, 3}, {3, 2}, {3, 3}, {4, 4}};
  const int ncand = (int)(sizeof cand / sizeof cand[0]);
  const int nu1_0 = ctx->nu1, nu2_0 = ctx->nu2;
  const bool timing_0 = ctx->timing;
  const bool have_force_0 = ctx->md_have_force;
  P3MZ_TRY(p3mz_set_timing(ctx, 1));
  // A frame's cycle count is the fractional count X at which the residual
  // crosses the threshold, rounded up; a few frames can show two schedules
  // with equal counts where one crosses just in time and the other with a
  // margin.  The expected count over a trajectory is E[ceil X] ~ mean X + 1/2
  // (fractional parts spread over [0, 1)), so each candidate's measured time
  // is corrected by (mean X + 1/2 - mean count) times its measured time per
  // cycle (one V-cycle plus the outer residual, launched back to back).
  // X interpolates log(residual) within the last cycle: with C cycles,
  // X = C - 1 + log(res[C-1] / thresh) / log(res[C-1] / res[C]).
  hipEvent_t c0, c1;
  P3MZ_HIP_TRY(hipEventCreate(&c0));
  P3MZ_HIP_TRY(hipEventCreate(&c1));
  int best = 0;
  for (int k = 0; k < ncand; k++) {
    P3MZ_TRY(p3mz_set_schedule(ctx, cand[k][0], cand[k][1], best_tile));
    double total = 0.0, xsum = 0.0;
    int cycles = 0;
    for (int pass = 0; pass < 2; pass++) {   // the first pass captures the graphs
      P3MZ_TRY(p3mz_load_state(ctx, blob.data(), bytes));
      total = 0.0;
      xsum = 0.0;
      cycles = 0;
      for (int f = 0; f < n_frames; f++) {
        p3mz_status st = compute_step(ctx, frames_dev + (size_t)3 * ctx->n_atoms * f, nullptr, nullptr, s);
        if (st < 0) return st;
        total += ctx->st.ms_mesh;
        const int C = ctx->st.cycles;
        cycles += C;
        double x = (double)C;
        if (C >= 1) {
          const double a = ctx->st.res_hist[C - 1], b = ctx->st.res_hist[C], t = ctx->st.thresh;
          if (a > t && b > 0.0 && b < a) x = (double)(C - 1) + std::min(1.0, std::log(a / t) / std::log(a / b));
        }
        xsum += x;
      }
    }
    // time per cycle: a V-cycle and the outer residual on the last frame's
    // level data (scratch of the step; the history is restored below)
    const LevelBufs& f0 = ctx->lv[0];
    const int reps = 4;
    float cyc_ms = 0.f;
    for (int pass = 0; pass < 2; pass++) {   // the first pass warms up
      P3MZ_HIP_TRY(hipEventRecord(c0, s));
      for (int r = 0; r < reps; r++) {
        P3MZ_HIP_TRY(launch_set_ctl_open(ctx->d_ctl, s));
        P3MZ_HIP_TRY(launch_vcycle(ctx->fp64, ctx->lv, ctx->pl.levels, ctx->pl.tail, ctx->nu1, ctx->nu2,
                                   ctx->d_green, ctx->d_ctl, s, nullptr));
        P3MZ_HIP_TRY(launch_outer(ctx->fp64, n, 0, ctx->P.max_cycles, ctx->d_sigma, ctx->d_y[0], ctx->d_y[1],
                                  cycle_e0(f0, ctx->fp64, ctx->nu2), cycle_e1(f0, ctx->fp64, ctx->nu2), f0.r0, f0.r1, ctx->d_partial, ctx->d_ctl, s, false, nullptr, 0.0, 0,
                                  ctx->P.stencil));
      }
      P3MZ_HIP_TRY(hipEventRecord(c1, s));
      P3MZ_HIP_TRY(hipEventSynchronize(c1));
      P3MZ_HIP_TRY(hipEventElapsedTime(&cyc_ms, c0, c1));
    }
    out->cand_nu_pre[k] = cand[k][0];
    out->cand_nu_post[k] = cand[k][1];
    out->cand_ms[k] = total / n_frames;
    out->cand_cycles[k] = cycles;
    out->cand_ms_cycle[k] = cyc_ms / reps;
    out->cand_cycles_frac[k] = xsum / n_frames;
    out->cand_expected_ms[k] =
        out->cand_ms[k] + out->cand_ms_cycle[k] * (out->cand_cycles_frac[k] + 0.5 - (double)cycles / n_frames);
    if (out->cand_expected_ms[k] < out->cand_expected_ms[best]) best = k;
  }
  (void)hipEventDestroy(c0);
  (void)hipEventDestroy(c1);
  out->n_candidates = ncand;
  out->nu_pre = cand[best][0];
  out->nu_post = cand[best][1];
  out->ms_best = out->cand_expected_ms[best];
  out->ms_default = out->cand_expected_ms[0];
  // restore the history, apply the choice and store it
  P3MZ_TRY(p3mz_load_state(ctx, blob.data(), bytes));
  P3MZ_TRY(p3mz_set_timing(ctx, timing_0));
  ctx->md_have_force = have_force_0 && nu1_0 == out->nu_pre && nu2_0 == out->nu_post;
  P3MZ_TRY(p3mz_set_schedule(ctx, out->nu_pre, out->nu_post, out->smooth_tile));
  TuneEntry t;
  t.nu_pre = out->nu_pre;
  t.nu_post = out->nu_post;
  t.smooth_tile = out->smooth_tile;
  t.ms = out->ms_best;
  return tune_store(tune_key(n, ctx->pl.p, ctx->P.precision), t);
}

void p3mz_destroy(p3mz_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free V-cycle.  The level hierarchy, the 4^3 Green's function and
// a control block of one V-cycle on a mesh of at most kNoallocMaxMesh points
// per edge live in a fixed device array.  Host code never uses the array's
// name as a device address: each device's copy is located once with
// hipGetSymbolAddress and that address is passed to the kernels.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoallocMaxMesh = 64;
constexpr size_t kNoallocBytes = 8u << 20;
constexpr int kNoallocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

struct NoallocDevice {
  unsigned char* base = nullptr;   // this device's copy of `scratch`
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc[kNoallocMaxDevices];

// Carves the level hierarchy of an n^3 mesh out of the scratch array (the
// same buffers a context allocates for p3mz_vcycle).  Returns the bytes used.
size_t noalloc_layout(unsigned char* base, int n, size_t ts, int levels, int tail, LevelBufs* lv, Ctl** ctl,
                      double** green) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return (void*)p;
  };
  *ctl = (Ctl*)take(sizeof(Ctl));
  *green = (double*)take(64 * sizeof(double));
  for (int l = 0; l < levels; l++) {
    const int nl = n >> l;
    const size_t half = (size_t)nl * nl * nl / 2;
    LevelBufs& b = lv[l];
    b = LevelBufs{};
    b.n = nl;
    b.e0 = take(half * ts);
    b.e1 = take(half * ts);
    b.r0 = take(half * ts);
    b.r1 = take(half * ts);
    if (l < tail && nl <= kFusedEdgeMax && nl >= 16) {
      b.d0 = take(half * ts);
      b.d1 = take(half * ts);
      b.fty = b.ftz = fused_tile(nl);
    }
  }
  return off;
}

// First call on the current device: locate its copy of the scratch array,
// store the Green's function there and allow the kernels their LDS.
p3mz_status noalloc_device(unsigned char** base) {
  int dev = 0;
  P3MZ_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocMaxDevices) return fail(P3MZ_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoallocDevice& d = g_noalloc[dev];
  if (!d.base) {
    void* ptr = nullptr;
    P3MZ_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    LevelBufs lv[P3MZ_MAX_LEVELS];
    Ctl* ctl = nullptr;
    double* green = nullptr;
    noalloc_layout((unsigned char*)ptr, 8, 8, 2, 0, lv, &ctl, &green);
    double g[64];
    coarse_green(g);
    P3MZ_HIP_TRY(hipMemcpy(green, g, sizeof g, hipMemcpyHostToDevice));
    size_t lds = 0;
    for (int fp64 = 0; fp64 < 2; fp64++) {
      P3MZ_HIP_TRY(tail_configure(fp64 != 0, 8, 2, &lds));
      P3MZ_HIP_TRY(tail_configure(fp64 != 0, 16, 3, &lds));
    }
    P3MZ_HIP_TRY(fused_configure());
    P3MZ_HIP_TRY(hipDeviceSynchronize());
    d.base = (unsigned char*)ptr;
  }
  *base = d.base;
  return P3MZ_OK;
}

}  // namespace

extern "C" {

p3mz_status p3mz_vcycle_noalloc(int32_t mesh, int32_t precision, int32_t nu_pre, int32_t nu_post, const double* r_dev,
                                double* e_dev, void* stream) {
  if (!r_dev || !e_dev) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  int m = mesh;
  while (m > 4 && (m & 1) == 0) m >>= 1;
  if (mesh < 8 || m != 4 || mesh > kNoallocMaxMesh)
    return fail(P3MZ_ERR_INVALID_ARG, "mesh must be 4*2^m points per edge, 8..64");
  if (precision != P3MZ_PREC_FP64 && precision != P3MZ_PREC_MIXED) return fail(P3MZ_ERR_INVALID_ARG, "bad precision");
  if (nu_pre < 0 || nu_post < 0 || nu_pre > 16 || nu_post > 16 || nu_pre + nu_post < 1)
    return fail(P3MZ_ERR_INVALID_ARG, "bad sweep counts");
  unsigned char* base = nullptr;
  P3MZ_TRY(noalloc_device(&base));
  const bool fp64 = precision == P3MZ_PREC_FP64;
  int levels = 0, tail = 0;
  for (int q = mesh; q >= 4; q >>= 1) levels++;
  while ((mesh >> tail) > P3MZ_TAIL_MAX) tail++;
  LevelBufs lv[P3MZ_MAX_LEVELS];
  Ctl* ctl = nullptr;
  double* green = nullptr;
  if (noalloc_layout(base, mesh, fp64 ? 8 : 4, levels, tail, lv, &ctl, &green) > kNoallocBytes)
    return fail(P3MZ_ERR_INVALID_ARG, "mesh too large for the scratch array");
  hipStream_t s = (hipStream_t)stream;
  P3MZ_HIP_TRY(launch_set_ctl_open(ctl, s));
  P3MZ_HIP_TRY(launch_nat_to_cs(fp64, mesh, r_dev, lv[0].r0, lv[0].r1, s));
  P3MZ_HIP_TRY(launch_vcycle(fp64, lv, levels, tail, nu_pre, nu_post, green, ctl, s));
  P3MZ_HIP_TRY(launch_cs_to_nat(fp64, mesh, lv[0].e0, lv[0].e1, e_dev, s));
  return P3MZ_OK;
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

const char* p3mz_version(void) { return "p3maze-gfx950 0.3"; }

p3mz_status p3mz_batch_create(int32_t n_sys, const p3mz_params* per_sys, const int64_t* n_atoms,
                              const double* charges_packed_host, p3mz_batch** out) {
  if (!out) return fail(P3MZ_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_sys < 1 || n_sys > 65535 || !per_sys || !n_atoms || !charges_packed_host)
    return fail(P3MZ_ERR_INVALID_ARG, "bad batch arguments");
  for (int r = 0; r < n_sys; r++)
    if (per_sys[r].precision != per_sys[0].precision)
      return fail(P3MZ_ERR_INVALID_ARG, "all systems of a batch need the same precision");
  p3mz_batch* b = new (std::nothrow) p3mz_batch();
  if (!b) return fail(P3MZ_ERR_OUT_OF_MEMORY, "batch allocation");
  int64_t off = 0;
  for (int r = 0; r < n_sys; r++) {
    p3mz_ctx* c = nullptr;
    p3mz_status st = p3mz_create(&per_sys[r], n_atoms[r], charges_packed_host + off, &c);
    if (st != P3MZ_OK) {
      delete b;
      return st;
    }
    b->sys.push_back(c);
    b->off.push_back(off);
    off += n_atoms[r];
  }
  b->n_total = off;
  b->fp64 = per_sys[0].precision == P3MZ_PREC_FP64;
  // In a batch the tails of many systems run side by side on different
  // compute units, so one more level (32^3, kept in global memory) is
  // worth moving into the single-workgroup tail: it saves five launches per
  // V-cycle.  The tail performs the same operations in the same order as
  // the separate launches, so results are unchanged.
  // The fused legs of the small levels trade redundant halo work for fewer
  // launches; side by side with other systems' launches a batch is bound by
  // throughput instead, so batched systems keep one launch per sweep.
  for (p3mz_ctx* c : b->sys) {
    // batched systems scan the cells every step (no neighbour lists)
    const p3mz_status st = nbr_configure(c, 0.0, 0);
    if (st != P3MZ_OK) {
      delete b;
      return st;
    }
    Plan& pl = c->pl;
    pl.tail = 0;
    while ((pl.n >> pl.tail) > P3MZ_TAIL_MAX_BATCH) pl.tail++;
    for (int l = 0; l < pl.levels; l++) c->lv[l].fty = c->lv[l].ftz = 0;
    size_t lds = 0;
    const hipError_t e = tail_configure(c->fp64, pl.n >> pl.tail, pl.levels - pl.tail, &lds);
    if (e != hipSuccess) {
      delete b;
      return hip_fail(e, "tail_configure", __FILE__, __LINE__);
    }
  }
  std::vector<Ctl*> ctls;
  for (p3mz_ctx* c : b->sys) ctls.push_back(c->d_ctl);
  auto bail = [&](p3mz_status st) {
    delete b;
    return st;
  };
#define P3MZ_BTRY(expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return bail(hip_fail(e_, #expr, __FILE__, __LINE__));      \
  } while (0)
  P3MZ_BTRY(hipMalloc((void**)&b->d_ctls, n_sys * sizeof(Ctl*)));
  P3MZ_BTRY(hipMemcpy(b->d_ctls, ctls.data(), n_sys * sizeof(Ctl*), hipMemcpyHostToDevice));
  P3MZ_BTRY(hipMalloc((void**)&b->d_ctl_all, n_sys * sizeof(Ctl)));
  P3MZ_BTRY(hipHostMalloc((void**)&b->h_ctl_all, n_sys * sizeof(Ctl), hipHostMallocDefault));
  P3MZ_BTRY(hipMalloc((void**)&b->d_head, 4 * sizeof(int)));
  P3MZ_BTRY(hipHostMalloc((void**)&b->h_head, 4 * sizeof(int), hipHostMallocDefault));
  P3MZ_BTRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
#undef P3MZ_BTRY
  *out = b;
  return P3MZ_OK;
}

p3mz_status p3mz_batch_compute(p3mz_batch* b, const double* pos_dev, double* force_dev, double* energies_dev,
                               void* stream) {
  if (!b || !pos_dev) return fail(P3MZ_ERR_INVALID_ARG, "batch or pos_dev is NULL");
  hipStream_t s = (hipStream_t)stream;
  b->md_have_force = false;
  P3MZ_TRY(batch_prepare_compute(b, pos_dev, force_dev, energies_dev, nullptr));
  bool nc = false;
  P3MZ_TRY(batch_step(b, &b->compute, s, false, false, &nc));
  if (nc) return fail(P3MZ_WARN_NOT_CONVERGED, "V-cycle cap reached before the tolerance in a batched system");
  return P3MZ_OK;
}

p3mz_status p3mz_batch_md_run(p3mz_batch* b, double* pos_dev, double* vel_dev, const double* mass_dev,
                              const p3mz_mdterms* terms, double dt, int32_t n_steps, double* energy_log_dev,
                              int32_t* cycles_log_dev, void* stream) {
  if (!b || !pos_dev || !vel_dev || !mass_dev || !terms || n_steps < 0 || !(dt > 0))
    return fail(P3MZ_ERR_INVALID_ARG, "bad batch md_run arguments");
  if (terms->model < 0 || terms->model > 2) return fail(P3MZ_ERR_INVALID_ARG, "unknown model");
  if (terms->model == 2)
    for (p3mz_ctx* c : b->sys)
      if (c->n_atoms % 3) return fail(P3MZ_ERR_INVALID_ARG, "the water model needs O,H,H triples");
  hipStream_t s = (hipStream_t)stream;
  const MdArgs m0 = md_args_for(terms, dt);
  bool nc = false;
  std::vector<uint64_t> force_key = {(uint64_t)(uintptr_t)pos_dev, (uint64_t)(uintptr_t)vel_dev,
                                     (uint64_t)(uintptr_t)mass_dev, (uint64_t)m0.model};
  for (double v : m0.p) force_key.push_back(bits(v));
  if (b->md_have_force && b->md_force_key != force_key) b->md_have_force = false;
  if (!b->md_have_force) {
    P3MZ_TRY(batch_prepare_compute(b, pos_dev, nullptr, nullptr, &m0));
    P3MZ_TRY(batch_step(b, &b->compute, s, false, true, &nc));
    b->md_have_force = true;
    b->md_force_key = force_key;
  }
  P3MZ_TRY(batch_prepare_md(b, pos_dev, vel_dev, mass_dev, m0, energy_log_dev, cycles_log_dev, n_steps));
  hipLaunchKernelGGL(k_batch_md_reset, dim3((b->sys.size() + 255) / 256), dim3(256), 0, s, b->d_ctls,
                     (int)b->sys.size());
  P3MZ_HIP_TRY(hipGetLastError());
  bool worst = false;
  for (int step = 0; step < n_steps; step++) {
    P3MZ_TRY(batch_step(b, &b->md, s, true, false, &nc));
    worst |= nc;
  }
  if (worst) return fail(P3MZ_WARN_NOT_CONVERGED, "V-cycle cap reached before the tolerance in a batched system");
  return P3MZ_OK;
}

p3mz_status p3mz_batch_step(p3mz_batch* b, double* pos_dev, double* vel_dev, const double* mass_dev,
                            const p3mz_mdterms* terms, double dt, double* force_dev, double* energies_dev,
                            int32_t* cycles_dev, void* stream) {
  if (!b) return fail(P3MZ_ERR_INVALID_ARG, "batch is NULL");
  const p3mz_status st = p3mz_batch_md_run(b, pos_dev, vel_dev, mass_dev, terms, dt, 1, nullptr, cycles_dev, stream);
  if (st < 0) return st;
  hipStream_t s = (hipStream_t)stream;
  for (size_t r = 0; r < b->sys.size(); r++) {
    const p3mz_ctx* c = b->sys[r];
    if (force_dev)
      P3MZ_HIP_TRY(hipMemcpyAsync(force_dev + 3 * b->off[r], c->d_md_force, sizeof(double) * 3 * (size_t)c->n_atoms,
                                  hipMemcpyDeviceToDevice, s));
    if (energies_dev)
      P3MZ_HIP_TRY(hipMemcpyAsync(energies_dev + 4 * r, c->d_energy, 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return st;
}

p3mz_status p3mz_batch_get_stats(const p3mz_batch* b, int32_t sys, p3mz_stats* out) {
  if (!b || !out || sys < 0 || sys >= (int)b->sys.size()) return fail(P3MZ_ERR_INVALID_ARG, "bad batch stats arguments");
  *out = b->sys[sys]->st;
  return P3MZ_OK;
}

p3mz_status p3mz_batch_set_timing(p3mz_batch* b, int32_t on) {
  if (!b) return fail(P3MZ_ERR_INVALID_ARG, "batch is NULL");
  if (on && !b->ev[0])
    for (hipEvent_t& e : b->ev) P3MZ_HIP_TRY(hipEventCreate(&e));
  b->timing = on != 0;
  b->ms_mesh = b->ms_sr = -1.0;
  return P3MZ_OK;
}

p3mz_status p3mz_batch_set_graphs(p3mz_batch* b, int32_t on) {
  if (!b) return fail(P3MZ_ERR_INVALID_ARG, "batch is NULL");
  P3MZ_HIP_TRY(hipDeviceSynchronize());
  for (BatchSet* x : {&b->compute, &b->md})
    for (GraphSlot& g : x->g) g.reset();
  b->use_graphs = on != 0;
  return P3MZ_OK;
}

p3mz_status p3mz_batch_get_timing(const p3mz_batch* b, double* ms_mesh, double* ms_short_range, int32_t* graphs) {
  if (!b || !ms_mesh || !ms_short_range || !graphs) return fail(P3MZ_ERR_INVALID_ARG, "NULL argument");
  *ms_mesh = b->ms_mesh;
  *ms_short_range = b->ms_sr;
  *graphs = b->ran_graphs;
  return P3MZ_OK;
}

p3mz_status p3mz_batch_kernel_bench(p3mz_batch* b, int32_t kernel_id, int32_t reps, void* stream, double* avg_ms,
                                    double* bytes_per_launch) {
  if (!b || !avg_ms || !bytes_per_launch || reps < 1) return fail(P3MZ_ERR_INVALID_ARG, "bad kernel_bench arguments");
  if (kernel_id != KT_HALFSWEEP && kernel_id != KT_SWEEP0 && kernel_id != KT_RESTRICT && kernel_id != KT_PROLONG &&
      kernel_id != KT_TAIL && kernel_id != P3MZ_KERNEL_PERSIST_HALFSWEEP)
    return fail(P3MZ_ERR_INVALID_ARG, "kernel family not available for batched timing");
  hipStream_t s = (hipStream_t)stream;
  if (kernel_id == P3MZ_KERNEL_PERSIST_HALFSWEEP) {
    // `reps` half-sweeps of every system in one persistent launch
    const int R = (int)b->sys.size();
    std::vector<const LevelBufs*> lv0(R);
    std::vector<Ctl*> ctls(R);
    double bytes = 0.0;
    for (int r = 0; r < R; r++) {
      p3mz_ctx* c = b->sys[r];
      lv0[r] = &c->lv[0];
      ctls[r] = c->d_ctl;
      const double n3 = (double)c->pl.n * c->pl.n * c->pl.n;
      bytes += 1.5 * (double)c->tsz * n3;
    }
    const int grid = persist_grid();
    if (grid < 1) return fail(P3MZ_ERR_HIP, "no occupancy for the persistent kernel");
    size_t sys_bytes = persist_sys_bytes(b->fp64, R);
    void* d_sys = nullptr;
    int* d_work = nullptr;
    P3MZ_HIP_TRY(hipMalloc(&d_sys, sys_bytes));
    P3MZ_HIP_TRY(hipMalloc(&d_work, sizeof(int) * (2 + (size_t)R * reps)));
    for (p3mz_ctx* c : b->sys) P3MZ_HIP_TRY(launch_set_ctl_open(c->d_ctl, s));
    hipEvent_t e0, e1;
    P3MZ_HIP_TRY(hipEventCreate(&e0));
    P3MZ_HIP_TRY(hipEventCreate(&e1));
    // a warm-up launch, then the timed one
    P3MZ_HIP_TRY(persist_halfsweeps(b->fp64, lv0.data(), ctls.data(), R, reps, d_sys, d_work, grid, s, &sys_bytes,
                                    true));
    P3MZ_HIP_TRY(hipEventRecord(e0, s));
    P3MZ_HIP_TRY(persist_halfsweeps(b->fp64, lv0.data(), ctls.data(), R, reps, d_sys, d_work, grid, s, &sys_bytes,
                                    false));
    P3MZ_HIP_TRY(hipEventRecord(e1, s));
    P3MZ_HIP_TRY(hipEventSynchronize(e1));
    int flags[2] = {0, 0};
    P3MZ_HIP_TRY(hipMemcpy(flags, d_work, sizeof flags, hipMemcpyDeviceToHost));
    float ms = 0.f;
    P3MZ_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P3MZ_HIP_TRY(hipFree(d_sys));
    P3MZ_HIP_TRY(hipFree(d_work));
    if (flags[1]) return fail(P3MZ_ERR_STATE, "a persistent-kernel wait gave up");
    *avg_ms = ms / reps;
    *bytes_per_launch = bytes;
    return P3MZ_OK;
  }
  // one batched launch of the family on every system's finest level
  BatchSet tmp;
  std::vector<unsigned char> args;
  double bytes = 0.0;
  P3MZ_TRY(batch_record(b, &tmp, 0, &args, [&](int r) -> p3mz_status {
    p3mz_ctx* c = b->sys[r];
    double by = 0.0;
    rec_key(1);
    hipError_t e = launch_vcycle_kernel(c->fp64, kernel_id, c->lv, c->pl.levels, c->pl.tail, c->nu1, c->nu2,
                                        c->d_green, c->d_ctl, nullptr, &by);
    if (e != hipSuccess) return fail(P3MZ_ERR_INVALID_ARG, "kernel not available on every system's mesh");
    bytes += by;
    return P3MZ_OK;
  }));
  P3MZ_TRY(batch_upload(&tmp, args));
  for (p3mz_ctx* c : b->sys) P3MZ_HIP_TRY(launch_set_ctl_open(c->d_ctl, s));
  hipEvent_t e0, e1;
  P3MZ_HIP_TRY(hipEventCreate(&e0));
  P3MZ_HIP_TRY(hipEventCreate(&e1));
  P3MZ_HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; r++)
    for (const BatchLaunch& L : tmp.q[0]) P3MZ_HIP_TRY(L.many((const char*)tmp.d_args + L.off, L.count, L.gx, L.lds, s));
  P3MZ_HIP_TRY(hipEventRecord(e1, s));
  P3MZ_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  P3MZ_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P3MZ_HIP_TRY(hipFree(tmp.d_args));
  *avg_ms = ms / reps;
  *bytes_per_launch = bytes;
  return P3MZ_OK;
}

void p3mz_batch_destroy(p3mz_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  delete b;
}

}  // extern "C"

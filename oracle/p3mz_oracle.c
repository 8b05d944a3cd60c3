/*
 * p3mz_oracle.c -- plain CPU FP64 reference of the P3MaZe mesh step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It is
 * written for a reader checking it against the paper, not for speed: each
 * operator is a direct loop over the mesh in natural (x-fastest) layout,
 * OpenMP only splits the outermost loop where every iteration writes its own
 * outputs, and every sum that feeds a result is taken serially in index
 * order.
 *
 * Readings taken where the paper is silent (listed with reasons in the
 * design notes of the repository):
 *   - Gaussian width and Ewald splitting: sigma = 1/(sqrt(2) alpha), which
 *     turns Eq. 6 into erfc(alpha r)/r and Eq. 7 into -alpha/sqrt(pi) Q^2.
 *   - Smoothing (Results, molten-salt protocol: "diffusion-based", linear
 *     cost): K explicit diffusion steps [nu, 1-2nu, nu] along x, then y, then
 *     z, adding a variance sigma_s^2 = sigma^2 - p h^2/6 per dimension.  The
 *     order-p B-spline carries variance p h^2/12 once in the assignment and
 *     once more in the force/energy interpolation, so a charge seen through
 *     the mesh carries exactly the Gaussian variance sigma^2 of Eq. 4.
 *     K = ceil(2 sigma_s^2 / h^2), nu = sigma_s^2 / (2 K h^2) <= 1/4.
 *   - Long-range energy: 1/2 sum_a Q_a (W * phi)(r_a), the point-charge
 *     reading of Eq. 14 under which Eqs. 5-7 add up to the Ewald energy.
 *   - Multigrid (the footnote on one iteration = one V-cycle): vertex-centred
 *     periodic coarsening by 2 down to 4^3, red-black Gauss-Seidel smoothing,
 *     full-weighting restriction (times 4 for the rediscretised coarse
 *     operator), trilinear prolongation, exact DFT solve on 4^3.
 *   - Tolerance: max|M y - sigma_p| <= tol * max|q^s| (mode 0) or <= tol.
 *   - History: the first step (or one after a reset) is a cold solve from
 *     phi = 0; its y is not a multiplier of a Verlet prediction and is not
 *     stored, so later steps ramp the predictor order with the number of
 *     stored warm multipliers.  The mesh potential is kept zero-mean.
 */
#include "p3mz_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define IDX(n, i, j, k) ((size_t)(i) + (size_t)(n) * ((size_t)(j) + (size_t)(n) * (size_t)(k)))

static int wrapi(long i, int n) {
  long r = i % n;
  return (int)(r < 0 ? r + n : r);
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

struct orc_state {
  orc_params P;
  orc_plan plan;
  int64_t n;
  double* Q;
  size_t n3;
  /* step arrays (finest level) */
  double *q, *qs, *sigma_p, *y, *y_start, *r, *e, *phi_p;
  /* history: phi^k, phi^{k-1}, stored warm multipliers (newest first) */
  double *phi_k, *phi_km1, *yh[3];
  int n_yh, have_hist;
  /* short-range subset: when sr_subset is set, pairs are summed only for
   * the atoms listed in sr_targets (all partners), see orc_set_sr_targets */
  int sr_subset;
  int64_t n_sr_targets;
  int64_t* sr_targets;
  /* per-level multigrid work arrays */
  double *rho[ORC_MAX_LEVELS], *rl[ORC_MAX_LEVELS], *el[ORC_MAX_LEVELS];
  orc_stats st;
  /* Langevin thermostat of the OVRVO scheme (gamma 0: none) and its step
   * counter */
  double th_gamma, th_kt;
  uint64_t th_seed;
  int64_t th_step;
};

/* ------------------------------------------------------------------------ */
/* Derived parameters.                                                       */
/* ------------------------------------------------------------------------ */
int orc_plan_make(const orc_params* p, orc_plan* pl) {
  if (!p || !pl) return ORC_ERR_INVALID_ARG;
  if (!(p->box > 0) || !(p->alpha > 0) || !(p->r_cut > 0) || p->r_cut > 0.5 * p->box)
    return ORC_ERR_INVALID_ARG;
  if (p->order < 2 || p->order > 7 || !(p->tol > 0) || p->max_cycles < 0 ||
      p->max_cycles > ORC_MAX_CYCLES || p->predictor < 0 || p->predictor > 3 ||
      p->nu_pre < 0 || p->nu_post < 0 || p->nu_pre + p->nu_post < 1 ||
      p->tol_mode < 0 || p->tol_mode > 1 || p->excl_group < 0 || p->stencil < 0 || p->stencil > 1)
    return ORC_ERR_INVALID_ARG;
  int n = p->mesh;
  if (n < 8) return ORC_ERR_MESH_SHAPE;
  int m4 = n;
  while (m4 > 4 && m4 % 2 == 0) m4 /= 2;
  if (m4 != 4) return ORC_ERR_MESH_SHAPE;   /* N = 4 * 2^m */
  memset(pl, 0, sizeof *pl);
  pl->h = p->box / n;
  pl->sigma = 1.0 / (sqrt(2.0) * p->alpha);
  pl->sigma_s2 = pl->sigma * pl->sigma - p->order * pl->h * pl->h / 6.0;
  if (!(pl->sigma_s2 > 0)) return ORC_ERR_MESH_SHAPE; /* mesh too coarse for sigma */
  /* K steps of weight nu = sigma_s^2 / (2 K h^2): nu <= 1/4 in general; for
   * the fourth-order discretisation nu <= 1/6, where the K-step diffusion
   * also matches the Gaussian's fourth cumulant up to O(h^4) (the quartic
   * term K nu (1/12 - nu/2) (k h)^4 of its symbol vanishes at nu = 1/6) */
  pl->K = (int)ceil((p->stencil == 1 ? 3.0 : 2.0) * pl->sigma_s2 / (pl->h * pl->h));
  if (pl->K < 1) pl->K = 1;
  pl->nu_smooth = pl->sigma_s2 / (2.0 * pl->K * pl->h * pl->h);
  int l = 0;
  for (int m = n; m >= 4; m /= 2) {
    if (l >= ORC_MAX_LEVELS) return ORC_ERR_MESH_SHAPE;
    pl->nl[l++] = m;
  }
  pl->levels = l;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Charge assignment (Theory: "cubic B-splines", generalised to order p).    */
/* ------------------------------------------------------------------------ */

/* Cardinal B-spline M_p supported on [0, p], by the Cox-de Boor recursion
 * M_1 = indicator of [0,1), M_p(x) = (x M_{p-1}(x) + (p-x) M_{p-1}(x-1))/(p-1). */
double orc_bspline(int p, double x) {
  if (p == 1) return (x >= 0.0 && x < 1.0) ? 1.0 : 0.0;
  return (x * orc_bspline(p - 1, x) + (p - x) * orc_bspline(p - 1, x - 1.0)) / (p - 1);
}

/* Mesh points and weights along one dimension for a particle at mesh
 * coordinate u in [0, n]: the p points nearest to u, weight
 * W(u - m) = M_p(u - m + p/2) (the B-spline centred on the particle). */
void orc_stencil_1d(int p, int n, double u, int32_t* idx, double* w) {
  long first = (p % 2 == 0) ? (long)floor(u) - p / 2 + 1 : (long)floor(u + 0.5) - (p - 1) / 2;
  for (int j = 0; j < p; j++) {
    long m = first + j;
    w[j] = orc_bspline(p, u - (double)m + 0.5 * p);
    idx[j] = wrapi(m, n);
  }
}

/* Mesh coordinate of a position: wrap into the box, then divide by h. */
static double mesh_coord(double x, double box, int n) {
  double s = x / box;
  s -= floor(s);
  return s * n;
}

/* q_m = sum_b Q_b W(r_b - r_m) over the periodic mesh. */
void orc_assign(int p, int n, double box, int64_t n_atoms, const double* pos,
                const double* q_atoms, double* q_mesh) {
  memset(q_mesh, 0, sizeof(double) * (size_t)n * n * n);
  for (int64_t a = 0; a < n_atoms; a++) {
    int32_t ix[8], iy[8], iz[8];
    double wx[8], wy[8], wz[8];
    orc_stencil_1d(p, n, mesh_coord(pos[3 * a + 0], box, n), ix, wx);
    orc_stencil_1d(p, n, mesh_coord(pos[3 * a + 1], box, n), iy, wy);
    orc_stencil_1d(p, n, mesh_coord(pos[3 * a + 2], box, n), iz, wz);
    for (int c = 0; c < p; c++)
      for (int b = 0; b < p; b++)
        for (int d = 0; d < p; d++)
          q_mesh[IDX(n, ix[d], iy[b], iz[c])] += q_atoms[a] * wx[d] * wy[b] * wz[c];
  }
}

/* ------------------------------------------------------------------------ */
/* Smoothing of the assigned charges (diffusion steps per dimension).        */
/* ------------------------------------------------------------------------ */
void orc_smooth(int n, int k_steps, double nu, double* v) {
  for (int dim = 0; dim < 3; dim++) {
#pragma omp parallel for
    for (int outer = 0; outer < n; outer++) {
      double* line = (double*)malloc(sizeof(double) * n);
      double* next = (double*)malloc(sizeof(double) * n);
      for (int inner = 0; inner < n; inner++) {
        for (int t = 0; t < n; t++) {
          size_t at = dim == 0 ? IDX(n, t, inner, outer)
                    : dim == 1 ? IDX(n, inner, t, outer) : IDX(n, inner, outer, t);
          line[t] = v[at];
        }
        for (int s = 0; s < k_steps; s++) {
          for (int t = 0; t < n; t++)
            next[t] = nu * line[wrapi(t - 1, n)] + (1.0 - 2.0 * nu) * line[t] +
                      nu * line[wrapi(t + 1, n)];
          double* sw = line; line = next; next = sw;
        }
        for (int t = 0; t < n; t++) {
          size_t at = dim == 0 ? IDX(n, t, inner, outer)
                    : dim == 1 ? IDX(n, inner, t, outer) : IDX(n, inner, outer, t);
          v[at] = line[t];
        }
      }
      free(line);
      free(next);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Mesh operators.  M/h^2 is the 7-point Laplacian (Theory, Eq. 10 and the   */
/* seven-point stencil named in the force discussion).                       */
/* ------------------------------------------------------------------------ */
static double nbr_sum(int n, const double* v, int i, int j, int k) {
  int im = wrapi(i - 1, n), ip = wrapi(i + 1, n);
  int jm = wrapi(j - 1, n), jp = wrapi(j + 1, n);
  int km = wrapi(k - 1, n), kp = wrapi(k + 1, n);
  return ((v[IDX(n, im, j, k)] + v[IDX(n, ip, j, k)]) + (v[IDX(n, i, jm, k)] + v[IDX(n, i, jp, k)])) +
         (v[IDX(n, i, j, km)] + v[IDX(n, i, j, kp)]);
}

void orc_apply_m(int n, const double* v, double* out) {
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++)
        out[IDX(n, i, j, k)] = nbr_sum(n, v, i, j, k) - 6.0 * v[IDX(n, i, j, k)];
}

/* Higher-order discretisation (the paper's remark after Eq. 21 that
 * Hermitian discretisations could replace the seven-point stencil): the
 * Mehrstellen scheme for the Laplacian, A phi = B f with
 *   A = (1/6) [2 (sum of the 6 face neighbours) + (sum of the 12 edge
 *       neighbours) - 24 (centre)]            (19-point Laplacian times h^2)
 *   B = (1/12) [(sum of the 6 face neighbours) + 6 (centre)]
 * which is fourth-order accurate: the symbol ratio B(k)/A(k) equals
 * -1/(k h)^2 up to O((k h)^4). */
void orc_apply_a19(int n, const double* v, double* out) {
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        int im = wrapi(i - 1, n), ip = wrapi(i + 1, n);
        int jm = wrapi(j - 1, n), jp = wrapi(j + 1, n);
        int km = wrapi(k - 1, n), kp = wrapi(k + 1, n);
        double faces = nbr_sum(n, v, i, j, k);
        double edges = (v[IDX(n, im, jm, k)] + v[IDX(n, ip, jm, k)] + v[IDX(n, im, jp, k)] + v[IDX(n, ip, jp, k)]) +
                       (v[IDX(n, im, j, km)] + v[IDX(n, ip, j, km)] + v[IDX(n, im, j, kp)] + v[IDX(n, ip, j, kp)]) +
                       (v[IDX(n, i, jm, km)] + v[IDX(n, i, jp, km)] + v[IDX(n, i, jm, kp)] + v[IDX(n, i, jp, kp)]);
        out[IDX(n, i, j, k)] = (2.0 * faces + edges - 24.0 * v[IDX(n, i, j, k)]) / 6.0;
      }
}

void orc_apply_b(int n, const double* v, double* out) {
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) out[IDX(n, i, j, k)] = (nbr_sum(n, v, i, j, k) + 6.0 * v[IDX(n, i, j, k)]) / 12.0;
}

/* One Gauss-Seidel half-sweep for M e = r over the points of one colour
 * (colour 0 = red = (i+j+k) even).  Points of one colour only couple to the
 * other colour, so the order inside the half-sweep does not matter. */
void orc_rbgs(int n, double* e, const double* r, int colour) {
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++)
        if (((i + j + k) & 1) == colour)
          e[IDX(n, i, j, k)] = (nbr_sum(n, e, i, j, k) - r[IDX(n, i, j, k)]) / 6.0;
}

/* Full-weighting restriction to the even fine points, times 4 because the
 * coarse operator is the same stencil on spacing 2h. */
void orc_restrict(int n, const double* rho, double* rc) {
  static const double w[3] = {0.25, 0.5, 0.25};
  int nc = n / 2;
#pragma omp parallel for
  for (int K = 0; K < nc; K++)
    for (int J = 0; J < nc; J++)
      for (int I = 0; I < nc; I++) {
        double s = 0.0;
        for (int c = -1; c <= 1; c++)
          for (int b = -1; b <= 1; b++)
            for (int a = -1; a <= 1; a++)
              s += w[a + 1] * w[b + 1] * w[c + 1] *
                   rho[IDX(n, wrapi(2 * I + a, n), wrapi(2 * J + b, n), wrapi(2 * K + c, n))];
        rc[IDX(nc, I, J, K)] = 4.0 * s;
      }
}

/* e += trilinear interpolation of the coarse correction ec (mesh nc). */
void orc_prolong_add(int nc, const double* ec, double* e) {
  int n = 2 * nc;
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        int ci[3][2];
        double cw[3][2];
        int cnt[3];
        int f[3] = {i, j, k};
        for (int d = 0; d < 3; d++) {
          if (f[d] % 2 == 0) {
            ci[d][0] = f[d] / 2; cw[d][0] = 1.0; cnt[d] = 1;
          } else {
            ci[d][0] = (f[d] - 1) / 2; ci[d][1] = wrapi((f[d] + 1) / 2, nc);
            cw[d][0] = 0.5; cw[d][1] = 0.5; cnt[d] = 2;
          }
        }
        double s = 0.0;
        for (int c = 0; c < cnt[2]; c++)
          for (int b = 0; b < cnt[1]; b++)
            for (int a = 0; a < cnt[0]; a++)
              s += cw[0][a] * cw[1][b] * cw[2][c] * ec[IDX(nc, ci[0][a], ci[1][b], ci[2][c])];
        e[IDX(n, i, j, k)] += s;
      }
}

/* Exact solve of M e = r on the periodic 4^3 mesh: M is diagonal in the
 * discrete Fourier basis with eigenvalue -sum_d 4 sin^2(pi k_d / 4); the
 * k = 0 mode (the null space) is set to zero, which also removes the mean
 * of r. */
void orc_coarsest(const double* r, double* e) {
  const int n = 4;
  double re[64], im[64];
  for (int kz = 0; kz < n; kz++)
    for (int ky = 0; ky < n; ky++)
      for (int kx = 0; kx < n; kx++) {
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < n; z++)
          for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
              double th = 2.0 * M_PI * (kx * x + ky * y + kz * z) / n;
              sr += r[IDX(n, x, y, z)] * cos(th);
              si -= r[IDX(n, x, y, z)] * sin(th);
            }
        size_t kk = IDX(n, kx, ky, kz);
        if (kx == 0 && ky == 0 && kz == 0) {
          re[kk] = 0.0; im[kk] = 0.0;
        } else {
          double sx = sin(M_PI * kx / n), sy = sin(M_PI * ky / n), sz = sin(M_PI * kz / n);
          double lam = -4.0 * (sx * sx + sy * sy + sz * sz);
          re[kk] = sr / lam; im[kk] = si / lam;
        }
      }
  for (int z = 0; z < n; z++)
    for (int y = 0; y < n; y++)
      for (int x = 0; x < n; x++) {
        double s = 0.0;
        for (int kz = 0; kz < n; kz++)
          for (int ky = 0; ky < n; ky++)
            for (int kx = 0; kx < n; kx++) {
              double th = 2.0 * M_PI * (kx * x + ky * y + kz * z) / n;
              size_t kk = IDX(n, kx, ky, kz);
              s += re[kk] * cos(th) - im[kk] * sin(th);
            }
        e[IDX(n, x, y, z)] = s / 64.0;
      }
}

/* One V-cycle for M e = r on level l, starting from e = 0 (footnote in the
 * performance section: relax, restrict, coarse-correct, prolong, relax). */
static void vcycle(orc_state* s, int l, const double* r, double* e) {
  const orc_plan* pl = &s->plan;
  int n = pl->nl[l];
  size_t n3 = (size_t)n * n * n;
  if (l == pl->levels - 1) {
    orc_coarsest(r, e);
    return;
  }
  memset(e, 0, sizeof(double) * n3);
  for (int it = 0; it < s->P.nu_pre; it++) {
    orc_rbgs(n, e, r, 0);
    orc_rbgs(n, e, r, 1);
  }
  double* rho = s->rho[l];
  orc_apply_m(n, e, rho);
  for (size_t t = 0; t < n3; t++) rho[t] = r[t] - rho[t];
  orc_restrict(n, rho, s->rl[l + 1]);
  vcycle(s, l + 1, s->rl[l + 1], s->el[l + 1]);
  orc_prolong_add(n / 2, s->el[l + 1], e);
  for (int it = 0; it < s->P.nu_post; it++) {
    orc_rbgs(n, e, r, 0);
    orc_rbgs(n, e, r, 1);
  }
}

int orc_vcycle_apply(orc_state* s, const double* r, double* e) {
  if (!s || !r || !e) return ORC_ERR_INVALID_ARG;
  vcycle(s, 0, r, e);
  return ORC_OK;
}

static double mean_of(const double* v, size_t n) {
  double acc = 0.0;
  for (size_t t = 0; t < n; t++) acc += v[t];
  return acc / (double)n;
}

static double maxabs_of(const double* v, size_t n) {
  double m = 0.0;
  for (size_t t = 0; t < n; t++) m = fmax(m, fabs(v[t]));
  return m;
}

/* ------------------------------------------------------------------------ */
/* Short-range pair term (Eqs. 6 and 20), minimum image, r < r_cut, with     */
/* the standard Ewald correction for excluded (intramolecular) pairs.        */
/* ------------------------------------------------------------------------ */
static double min_image(double d, double box) { return d - box * nearbyint(d / box); }

void orc_sr(int64_t n_atoms, const double* pos, const double* q, double box, double alpha,
            double r_cut, double k_e, int32_t excl_group, const int64_t* targets,
            int64_t n_targets, double* force, double* e_atom) {
  const double two_a_sqrtpi = 2.0 * alpha / sqrt(M_PI);
  const double rc2 = r_cut * r_cut;
  int64_t nt = targets ? n_targets : n_atoms;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nt; t++) {
    int64_t i = targets ? targets[t] : t;
    double fx = 0, fy = 0, fz = 0, en = 0;
    for (int64_t j = 0; j < n_atoms; j++) {
      if (j == i) continue;
      double dx = min_image(pos[3 * i] - pos[3 * j], box);
      double dy = min_image(pos[3 * i + 1] - pos[3 * j + 1], box);
      double dz = min_image(pos[3 * i + 2] - pos[3 * j + 2], box);
      double r2 = dx * dx + dy * dy + dz * dz;
      double r = sqrt(r2);
      double qq = k_e * q[i] * q[j];
      if (excl_group > 0 && i / excl_group == j / excl_group) {
        /* excluded pair: remove the part the mesh carries, -erf(alpha r)/r */
        double er = erf(alpha * r);
        double f = qq * (two_a_sqrtpi * exp(-alpha * alpha * r2) / r - er / r2) / r;
        fx += f * dx; fy += f * dy; fz += f * dz;
        en += -0.5 * qq * er / r;
        continue;
      }
      if (r2 >= rc2) continue;
      double ec = erfc(alpha * r);
      double f = qq * (ec / (r2 * r) + two_a_sqrtpi * exp(-alpha * alpha * r2) / r2);
      fx += f * dx; fy += f * dy; fz += f * dz;
      en += 0.5 * qq * ec / r;
    }
    if (force) { force[3 * t] = fx; force[3 * t + 1] = fy; force[3 * t + 2] = fz; }
    if (e_atom) e_atom[t] = en;
  }
}

/* ------------------------------------------------------------------------ */
/* Brute-force Ewald sum (test reference for the whole decomposition):       */
/* real-space erfc images + reciprocal sum + self term, each truncated where */
/* its terms fall below eps.                                                 */
/* ------------------------------------------------------------------------ */
int orc_ewald(int64_t n_atoms, const double* pos, const double* q, double box, double alpha,
              double k_e, double eps, double* energy3, double* force) {
  if (n_atoms <= 0 || !(box > 0) || !(alpha > 0)) return ORC_ERR_INVALID_ARG;
  double x = 1.0;
  while (erfc(x) > eps) x += 0.1;          /* erfc(alpha r_max) < eps */
  double r_max = x / alpha;
  int nimg = (int)ceil(r_max / box) + 1;
  double kx_max = 2.0 * alpha * sqrt(-log(eps));   /* exp(-k^2/(4a^2)) < eps */
  int mmax = (int)ceil(kx_max * box / (2.0 * M_PI));
  double vol = box * box * box;
  double e_real = 0.0, e_rec = 0.0, e_self = 0.0;
  double* f_real = (double*)calloc(3 * (size_t)n_atoms, sizeof(double));
  double* f_rec = (double*)calloc(3 * (size_t)n_atoms, sizeof(double));
  double* e_i = (double*)calloc((size_t)n_atoms, sizeof(double));
  if (!f_real || !f_rec || !e_i) { free(f_real); free(f_rec); free(e_i); return ORC_ERR_OUT_OF_MEMORY; }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_atoms; i++) {
    double acc = 0.0;
    for (int64_t j = 0; j < n_atoms; j++)
      for (int nz = -nimg; nz <= nimg; nz++)
        for (int ny = -nimg; ny <= nimg; ny++)
          for (int nx = -nimg; nx <= nimg; nx++) {
            if (i == j && nx == 0 && ny == 0 && nz == 0) continue;
            double dx = pos[3 * i] - pos[3 * j] + nx * box;
            double dy = pos[3 * i + 1] - pos[3 * j + 1] + ny * box;
            double dz = pos[3 * i + 2] - pos[3 * j + 2] + nz * box;
            double r2 = dx * dx + dy * dy + dz * dz;
            double r = sqrt(r2);
            if (r > r_max) continue;
            double ec = erfc(alpha * r);
            acc += 0.5 * q[i] * q[j] * ec / r;
            double f = q[i] * q[j] * (ec / r + 2.0 * alpha / sqrt(M_PI) * exp(-alpha * alpha * r2)) / r2;
            f_real[3 * i] += f * dx; f_real[3 * i + 1] += f * dy; f_real[3 * i + 2] += f * dz;
          }
    e_i[i] = acc;
  }
  for (int64_t i = 0; i < n_atoms; i++) e_real += e_i[i];
  /* reciprocal: (2 pi / V) sum_{k != 0} exp(-k^2/4a^2)/k^2 |S(k)|^2 */
  for (int mz = -mmax; mz <= mmax; mz++)
    for (int my = -mmax; my <= mmax; my++)
      for (int mx = -mmax; mx <= mmax; mx++) {
        if (mx == 0 && my == 0 && mz == 0) continue;
        double kx = 2.0 * M_PI * mx / box, ky = 2.0 * M_PI * my / box, kz = 2.0 * M_PI * mz / box;
        double k2 = kx * kx + ky * ky + kz * kz;
        double g = exp(-k2 / (4.0 * alpha * alpha)) / k2;
        if (g < eps * 1e-3) continue;
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n_atoms; j++) {
          double th = kx * pos[3 * j] + ky * pos[3 * j + 1] + kz * pos[3 * j + 2];
          sr += q[j] * cos(th);
          si += q[j] * sin(th);
        }
        e_rec += 2.0 * M_PI / vol * g * (sr * sr + si * si);
        for (int64_t i = 0; i < n_atoms; i++) {
          double th = kx * pos[3 * i] + ky * pos[3 * i + 1] + kz * pos[3 * i + 2];
          /* Im(S* e^{i k r_i}) = sr sin(th) - si cos(th) */
          double im = sr * sin(th) - si * cos(th);
          double f = 4.0 * M_PI / vol * g * q[i] * im;
          f_rec[3 * i] += f * kx; f_rec[3 * i + 1] += f * ky; f_rec[3 * i + 2] += f * kz;
        }
      }
  for (int64_t i = 0; i < n_atoms; i++) e_self -= alpha / sqrt(M_PI) * q[i] * q[i];
  energy3[0] = k_e * e_real;
  energy3[1] = k_e * e_rec;
  energy3[2] = k_e * e_self;
  if (force)
    for (size_t t = 0; t < 3 * (size_t)n_atoms; t++) force[t] = k_e * (f_real[t] + f_rec[t]);
  free(f_real); free(f_rec); free(e_i);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* State.                                                                    */
/* ------------------------------------------------------------------------ */
static double* alloc_mesh(size_t n) { return (double*)calloc(n, sizeof(double)); }

void orc_destroy(orc_state* s) {
  if (!s) return;
  free(s->Q); free(s->q); free(s->qs); free(s->sigma_p); free(s->y); free(s->y_start);
  free(s->r); free(s->e); free(s->phi_p); free(s->phi_k); free(s->phi_km1);
  for (int t = 0; t < 3; t++) free(s->yh[t]);
  for (int l = 0; l < ORC_MAX_LEVELS; l++) { free(s->rho[l]); free(s->rl[l]); free(s->el[l]); }
  free(s->sr_targets);
  free(s);
}

int orc_set_sr_targets(orc_state* s, const int64_t* targets, int64_t n_targets) {
  if (!s || n_targets < -1 || (n_targets > 0 && !targets)) return ORC_ERR_INVALID_ARG;
  for (int64_t t = 0; t < n_targets; t++)
    if (targets[t] < 0 || targets[t] >= s->n) return ORC_ERR_INVALID_ARG;
  free(s->sr_targets);
  s->sr_targets = NULL;
  s->n_sr_targets = 0;
  s->sr_subset = n_targets >= 0;
  if (n_targets > 0) {
    s->sr_targets = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_targets);
    if (!s->sr_targets) return ORC_ERR_OUT_OF_MEMORY;
    memcpy(s->sr_targets, targets, sizeof(int64_t) * (size_t)n_targets);
    s->n_sr_targets = n_targets;
  }
  return ORC_OK;
}

int orc_create(const orc_params* p, int64_t n_atoms, const double* charges, orc_state** out) {
  if (!p || !out || n_atoms < 1 || !charges) return ORC_ERR_INVALID_ARG;
  *out = NULL;
  orc_plan pl;
  int rc = orc_plan_make(p, &pl);
  if (rc) return rc;
  /* the periodic problem is solvable only for a neutral system */
  double sq = 0.0, sa = 0.0;
  for (int64_t a = 0; a < n_atoms; a++) { sq += charges[a]; sa += fabs(charges[a]); }
  if (fabs(sq) > 1e-10 * sa) return ORC_ERR_NOT_NEUTRAL;
  orc_state* s = (orc_state*)calloc(1, sizeof *s);
  if (!s) return ORC_ERR_OUT_OF_MEMORY;
  s->P = *p;
  s->plan = pl;
  s->n = n_atoms;
  s->n3 = (size_t)p->mesh * p->mesh * p->mesh;
  s->Q = (double*)malloc(sizeof(double) * n_atoms);
  if (s->Q) memcpy(s->Q, charges, sizeof(double) * n_atoms);
  s->q = alloc_mesh(s->n3); s->qs = alloc_mesh(s->n3); s->sigma_p = alloc_mesh(s->n3);
  s->y = alloc_mesh(s->n3); s->y_start = alloc_mesh(s->n3); s->r = alloc_mesh(s->n3);
  s->e = alloc_mesh(s->n3); s->phi_p = alloc_mesh(s->n3); s->phi_k = alloc_mesh(s->n3); s->phi_km1 = alloc_mesh(s->n3);
  int ok = s->Q && s->q && s->qs && s->sigma_p && s->y && s->y_start && s->r && s->e && s->phi_p &&
           s->phi_k && s->phi_km1;
  for (int t = 0; t < 3; t++) { s->yh[t] = alloc_mesh(s->n3); ok = ok && s->yh[t]; }
  for (int l = 0; l < pl.levels; l++) {
    size_t m = (size_t)pl.nl[l] * pl.nl[l] * pl.nl[l];
    s->rho[l] = alloc_mesh(m); s->rl[l] = alloc_mesh(m); s->el[l] = alloc_mesh(m);
    ok = ok && s->rho[l] && s->rl[l] && s->el[l];
  }
  if (!ok) { orc_destroy(s); return ORC_ERR_OUT_OF_MEMORY; }
  *out = s;
  return ORC_OK;
}

int orc_reset_history(orc_state* s) {
  if (!s) return ORC_ERR_INVALID_ARG;
  s->have_hist = 0;
  s->n_yh = 0;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One mesh step.                                                            */
/* ------------------------------------------------------------------------ */
int orc_compute(orc_state* s, const double* pos, double* force, double* energy4) {
  if (!s || !pos) return ORC_ERR_INVALID_ARG;
  const orc_params* P = &s->P;
  const orc_plan* pl = &s->plan;
  const int n = P->mesh, p = P->order;
  const size_t n3 = s->n3;
  const double h = pl->h;
  for (int64_t t = 0; t < 3 * s->n; t++)
    if (!isfinite(pos[t])) return ORC_ERR_INVALID_ARG;

  double t0 = now_s();
  /* assignment, then smoothing to q^s */
  orc_assign(p, n, P->box, s->n, pos, s->Q, s->q);
  memcpy(s->qs, s->q, sizeof(double) * n3);
  orc_smooth(n, pl->K, pl->nu_smooth, s->qs);
  double t1 = now_s();

  /* Verlet prediction phi_p = 2 phi^k - phi^{k-1} (zero on a cold solve) and
   * the constraint at the prediction, sigma_p = (h/4pi) M phi_p + q^s (Eq. 17),
   * projected to zero mean.  With the fourth-order discretisation the
   * constraint is A phi = -(4 pi / h) B q^s, so sigma_p = (h/4pi) A phi_p +
   * B q^s and the correction problem below is A y = sigma_p. */
  const int ho = P->stencil == 1;
  const int cold = !s->have_hist;
  double* phi_p = s->phi_p;
  if (cold) {
    memset(phi_p, 0, sizeof(double) * n3);
  } else {
    for (size_t t = 0; t < n3; t++) phi_p[t] = 2.0 * s->phi_k[t] - s->phi_km1[t];
  }
  if (ho) {
    orc_apply_a19(n, phi_p, s->sigma_p);
    orc_apply_b(n, s->qs, s->r);   /* B q^s, r is free here */
    for (size_t t = 0; t < n3; t++) s->sigma_p[t] = h / (4.0 * M_PI) * s->sigma_p[t] + s->r[t];
  } else {
    orc_apply_m(n, phi_p, s->sigma_p);
    for (size_t t = 0; t < n3; t++) s->sigma_p[t] = h / (4.0 * M_PI) * s->sigma_p[t] + s->qs[t];
  }
  double ms = mean_of(s->sigma_p, n3);
  for (size_t t = 0; t < n3; t++) s->sigma_p[t] -= ms;

  /* multiplier predictor (Results, water convergence discussion):
   * y0 = y^k, 2y^k - y^{k-1}, or 3y^k - 3y^{k-1} + y^{k-2} */
  int m_eff = cold ? 0 : (P->predictor < s->n_yh ? P->predictor : s->n_yh);
  for (size_t t = 0; t < n3; t++) {
    double v = 0.0;
    if (m_eff == 1) v = s->yh[0][t];
    else if (m_eff == 2) v = 2.0 * s->yh[0][t] - s->yh[1][t];
    else if (m_eff == 3) v = 3.0 * s->yh[0][t] - 3.0 * s->yh[1][t] + s->yh[2][t];
    s->y[t] = v;
  }
  memcpy(s->y_start, s->y, sizeof(double) * n3);

  /* correction problem M y = sigma_p (Eq. 16) by V-cycles; the residual
   * max|M y - sigma_p| (Eq. 26) is tested before every cycle.  For the
   * fourth-order operator A the residual uses A and each V-cycle (on the
   * seven-point M) gives the correction: defect correction, which
   * converges because A and M agree on the smooth modes that carry the
   * Gaussian-smoothed charge. */
  double norm = maxabs_of(s->qs, n3);
  double thresh = P->tol_mode == 0 ? P->tol * norm : P->tol;
  int cycles = 0, status = ORC_OK;
  for (;;) {
    if (ho)
      orc_apply_a19(n, s->y, s->r);
    else
      orc_apply_m(n, s->y, s->r);
    for (size_t t = 0; t < n3; t++) s->r[t] = s->sigma_p[t] - s->r[t];
    double res = maxabs_of(s->r, n3);
    s->st.res_hist[cycles] = res;
    if (res <= thresh) break;
    if (cycles == P->max_cycles) { status = ORC_WARN_NOT_CONVERGED; break; }
    vcycle(s, 0, s->r, s->e);
    for (size_t t = 0; t < n3; t++) s->y[t] += s->e[t];
    cycles++;
  }
  double my = mean_of(s->y, n3);
  for (size_t t = 0; t < n3; t++) s->y[t] -= my;

  /* field update phi^{k+1} = phi_p - (4 pi / h) y (Supporting Information,
   * numerical integration) and history rotation */
  for (size_t t = 0; t < n3; t++) s->phi_km1[t] = phi_p[t] - 4.0 * M_PI / h * s->y[t];
  /* phi_km1 now holds phi^{k+1}; swap so phi_k is the newest field */
  double* sw = s->phi_k; s->phi_k = s->phi_km1; s->phi_km1 = sw;
  if (cold) {
    memcpy(s->phi_km1, s->phi_k, sizeof(double) * n3);
    s->n_yh = 0;
  } else {
    double* oldest = s->yh[2];
    s->yh[2] = s->yh[1]; s->yh[1] = s->yh[0]; s->yh[0] = oldest;
    memcpy(s->yh[0], s->y, sizeof(double) * n3);
    if (s->n_yh < 3) s->n_yh++;
  }
  s->have_hist = 1;
  double t2 = now_s();

  /* long-range force (Eq. 21): -Q sum_n W(r - r_n) (D phi)_n with the
   * central difference D (two-point; four-point, fourth order, with the
   * Mehrstellen Laplacian), and the long-range energy 1/2 Q (W * phi)(r) */
  const double* phi = s->phi_k;
  double* e_at = (double*)malloc(sizeof(double) * (size_t)s->n);
  if (!e_at) return ORC_ERR_OUT_OF_MEMORY;
#pragma omp parallel for
  for (int64_t a = 0; a < s->n; a++) {
    int32_t ix[8], iy[8], iz[8];
    double wx[8], wy[8], wz[8];
    orc_stencil_1d(p, n, mesh_coord(pos[3 * a + 0], P->box, n), ix, wx);
    orc_stencil_1d(p, n, mesh_coord(pos[3 * a + 1], P->box, n), iy, wy);
    orc_stencil_1d(p, n, mesh_coord(pos[3 * a + 2], P->box, n), iz, wz);
    double gx = 0, gy = 0, gz = 0, pot = 0;
    for (int c = 0; c < p; c++)
      for (int b = 0; b < p; b++)
        for (int d = 0; d < p; d++) {
          int i = ix[d], j = iy[b], k = iz[c];
          double W = wx[d] * wy[b] * wz[c];
          double dx, dy, dz;
          if (ho) {
            /* (8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2})) / (12 h) */
            dx = (8.0 * (phi[IDX(n, wrapi(i + 1, n), j, k)] - phi[IDX(n, wrapi(i - 1, n), j, k)]) -
                  (phi[IDX(n, wrapi(i + 2, n), j, k)] - phi[IDX(n, wrapi(i - 2, n), j, k)])) / (12.0 * h);
            dy = (8.0 * (phi[IDX(n, i, wrapi(j + 1, n), k)] - phi[IDX(n, i, wrapi(j - 1, n), k)]) -
                  (phi[IDX(n, i, wrapi(j + 2, n), k)] - phi[IDX(n, i, wrapi(j - 2, n), k)])) / (12.0 * h);
            dz = (8.0 * (phi[IDX(n, i, j, wrapi(k + 1, n))] - phi[IDX(n, i, j, wrapi(k - 1, n))]) -
                  (phi[IDX(n, i, j, wrapi(k + 2, n))] - phi[IDX(n, i, j, wrapi(k - 2, n))])) / (12.0 * h);
          } else {
            dx = (phi[IDX(n, wrapi(i + 1, n), j, k)] - phi[IDX(n, wrapi(i - 1, n), j, k)]) / (2.0 * h);
            dy = (phi[IDX(n, i, wrapi(j + 1, n), k)] - phi[IDX(n, i, wrapi(j - 1, n), k)]) / (2.0 * h);
            dz = (phi[IDX(n, i, j, wrapi(k + 1, n))] - phi[IDX(n, i, j, wrapi(k - 1, n))]) / (2.0 * h);
          }
          gx += W * dx; gy += W * dy; gz += W * dz;
          pot += W * phi[IDX(n, i, j, k)];
        }
    if (force) {
      force[3 * a + 0] = -P->coulomb_k * s->Q[a] * gx;
      force[3 * a + 1] = -P->coulomb_k * s->Q[a] * gy;
      force[3 * a + 2] = -P->coulomb_k * s->Q[a] * gz;
    }
    e_at[a] = 0.5 * P->coulomb_k * s->Q[a] * pot;
  }
  double e_lr = 0.0;
  for (int64_t a = 0; a < s->n; a++) e_lr += e_at[a];
  double t3 = now_s();

  /* short-range pairs (Eqs. 6, 20) and the Gaussian self term (Eq. 7) */
  double* f_sr = (double*)malloc(sizeof(double) * 3 * (size_t)s->n);
  if (!f_sr) { free(e_at); return ORC_ERR_OUT_OF_MEMORY; }
  double e_sr = 0.0, e_self = 0.0;
  if (s->sr_subset) {
    memset(f_sr, 0, sizeof(double) * 3 * (size_t)s->n);
    if (s->n_sr_targets > 0) {
      const int64_t nt = s->n_sr_targets;
      double* ft = (double*)malloc(sizeof(double) * 3 * (size_t)nt);
      if (!ft) { free(f_sr); free(e_at); return ORC_ERR_OUT_OF_MEMORY; }
      orc_sr(s->n, pos, s->Q, P->box, P->alpha, P->r_cut, P->coulomb_k, P->excl_group, s->sr_targets, nt, ft,
             NULL);
      for (int64_t t = 0; t < nt; t++)
        for (int d = 0; d < 3; d++) f_sr[3 * s->sr_targets[t] + d] = ft[3 * t + d];
      free(ft);
    }
    e_sr = NAN;   /* only a subset of the pair sum was formed */
  } else {
    orc_sr(s->n, pos, s->Q, P->box, P->alpha, P->r_cut, P->coulomb_k, P->excl_group, NULL, 0, f_sr, e_at);
    for (int64_t a = 0; a < s->n; a++) e_sr += e_at[a];
  }
  for (int64_t a = 0; a < s->n; a++) e_self -= P->coulomb_k * P->alpha / sqrt(M_PI) * s->Q[a] * s->Q[a];
  if (force)
    for (size_t t = 0; t < 3 * (size_t)s->n; t++) force[t] += f_sr[t];
  free(f_sr);
  free(e_at);
  double t4 = now_s();

  s->st.status = status;
  s->st.cycles = cycles;
  s->st.cold = cold;
  s->st.m_eff = m_eff;
  s->st.thresh = thresh;
  s->st.norm_qs = norm;
  s->st.e_sr = e_sr;
  s->st.e_lr = e_lr;
  s->st.e_self = e_self;
  s->st.e_total = e_sr + e_lr + e_self;
  s->st.t_spread = t1 - t0;
  s->st.t_solve = t2 - t1;
  s->st.t_gather = t3 - t2;
  s->st.t_sr = t4 - t3;
  s->st.steps++;
  if (energy4) {
    energy4[0] = e_sr; energy4[1] = e_lr; energy4[2] = e_self; energy4[3] = s->st.e_total;
  }
  return status;
}

int orc_get_stats(const orc_state* s, orc_stats* out) {
  if (!s || !out) return ORC_ERR_INVALID_ARG;
  *out = s->st;
  return ORC_OK;
}

int orc_get_plan(const orc_state* s, orc_plan* out) {
  if (!s || !out) return ORC_ERR_INVALID_ARG;
  *out = s->plan;
  return ORC_OK;
}

int orc_get_mesh(const orc_state* s, int which, double* out) {
  if (!s || !out) return ORC_ERR_INVALID_ARG;
  const double* src = NULL;
  switch (which) {
    case ORC_MESH_Q: src = s->q; break;
    case ORC_MESH_QS: src = s->qs; break;
    case ORC_MESH_SIGMA_P: src = s->sigma_p; break;
    case ORC_MESH_Y: src = s->y; break;
    case ORC_MESH_PHI: src = s->phi_k; break;
    case ORC_MESH_PHI_PREV: src = s->phi_km1; break;
    case ORC_MESH_Y_START: src = s->y_start; break;
    default: return ORC_ERR_INVALID_ARG;
  }
  memcpy(out, src, sizeof(double) * s->n3);
  return ORC_OK;
}

/* state = {have_hist, n_yh, steps, phi^k, phi^{k-1}, yh[0..2]} */
int orc_save_state(const orc_state* s, void* buf, size_t* bytes) {
  if (!s || !bytes) return ORC_ERR_INVALID_ARG;
  size_t need = 3 * sizeof(int64_t) + 5 * s->n3 * sizeof(double);
  if (!buf) { *bytes = need; return ORC_OK; }
  if (*bytes < need) return ORC_ERR_INVALID_ARG;
  int64_t hdr[3] = {s->have_hist, s->n_yh, s->st.steps};
  char* c = (char*)buf;
  memcpy(c, hdr, sizeof hdr); c += sizeof hdr;
  const double* arr[5] = {s->phi_k, s->phi_km1, s->yh[0], s->yh[1], s->yh[2]};
  for (int t = 0; t < 5; t++) { memcpy(c, arr[t], s->n3 * sizeof(double)); c += s->n3 * sizeof(double); }
  *bytes = need;
  return ORC_OK;
}

int orc_load_state(orc_state* s, const void* buf, size_t bytes) {
  if (!s || !buf) return ORC_ERR_INVALID_ARG;
  size_t need = 3 * sizeof(int64_t) + 5 * s->n3 * sizeof(double);
  if (bytes != need) return ORC_ERR_INVALID_ARG;
  int64_t hdr[3];
  const char* c = (const char*)buf;
  memcpy(hdr, c, sizeof hdr); c += sizeof hdr;
  s->have_hist = (int)hdr[0]; s->n_yh = (int)hdr[1]; s->st.steps = hdr[2];
  double* arr[5] = {s->phi_k, s->phi_km1, s->yh[0], s->yh[1], s->yh[2]};
  for (int t = 0; t < 5; t++) { memcpy(arr[t], c, s->n3 * sizeof(double)); c += s->n3 * sizeof(double); }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Non-electrostatic terms for the molecular-dynamics checks.                */
/* ------------------------------------------------------------------------ */
int orc_nonelectrostatic(const orc_mdterms* t, int64_t n_atoms, const double* pos, double box,
                         double r_cut, double* force, double* energy) {
  memset(force, 0, sizeof(double) * 3 * (size_t)n_atoms);
  *energy = 0.0;
  if (!t || t->model == 0) return ORC_OK;
  double* e_at = (double*)calloc((size_t)n_atoms, sizeof(double));
  if (!e_at) return ORC_ERR_OUT_OF_MEMORY;
  const double rc2 = r_cut * r_cut;
  if (t->model == 1) {
    /* stand-in Born-Mayer repulsion A exp(-r/rho), shifted to zero at r_cut */
    double shift = t->bm_a * exp(-r_cut / t->bm_rho);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_atoms; i++) {
      double fx = 0, fy = 0, fz = 0, en = 0;
      for (int64_t j = 0; j < n_atoms; j++) {
        if (j == i) continue;
        double dx = min_image(pos[3 * i] - pos[3 * j], box);
        double dy = min_image(pos[3 * i + 1] - pos[3 * j + 1], box);
        double dz = min_image(pos[3 * i + 2] - pos[3 * j + 2], box);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rc2) continue;
        double r = sqrt(r2);
        double v = t->bm_a * exp(-r / t->bm_rho);
        double f = v / t->bm_rho / r;
        fx += f * dx; fy += f * dy; fz += f * dz;
        en += 0.5 * (v - shift);
      }
      force[3 * i] = fx; force[3 * i + 1] = fy; force[3 * i + 2] = fz;
      e_at[i] = en;
    }
  } else if (t->model == 2) {
    /* flexible water, atoms O,H,H per molecule: intermolecular O-O
     * Lennard-Jones (shifted to zero at r_cut), harmonic bonds and angle */
    double sr6c = pow(t->lj_sigma * t->lj_sigma / rc2, 3);
    double shift = 4.0 * t->lj_eps * (sr6c * sr6c - sr6c);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_atoms; i += 3) {
      double fx = 0, fy = 0, fz = 0, en = 0;
      for (int64_t j = 0; j < n_atoms; j += 3) {
        if (j == i) continue;
        double dx = min_image(pos[3 * i] - pos[3 * j], box);
        double dy = min_image(pos[3 * i + 1] - pos[3 * j + 1], box);
        double dz = min_image(pos[3 * i + 2] - pos[3 * j + 2], box);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rc2) continue;
        double sr2 = t->lj_sigma * t->lj_sigma / r2;
        double sr6 = sr2 * sr2 * sr2;
        double f = 24.0 * t->lj_eps * (2.0 * sr6 * sr6 - sr6) / r2;
        fx += f * dx; fy += f * dy; fz += f * dz;
        en += 0.5 * (4.0 * t->lj_eps * (sr6 * sr6 - sr6) - shift);
      }
      force[3 * i] = fx; force[3 * i + 1] = fy; force[3 * i + 2] = fz;
      e_at[i] = en;
    }
    for (int64_t o = 0; o + 2 < n_atoms; o += 3) {
      double a[3], b[3];
      for (int d = 0; d < 3; d++) {
        a[d] = min_image(pos[3 * (o + 1) + d] - pos[3 * o + d], box);
        b[d] = min_image(pos[3 * (o + 2) + d] - pos[3 * o + d], box);
      }
      double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      /* bonds: V = 0.5 k (r - r0)^2, force on H = -k (r - r0) r_hat */
      double fa = -t->k_bond * (la - t->r0) / la, fb = -t->k_bond * (lb - t->r0) / lb;
      double en = 0.5 * t->k_bond * ((la - t->r0) * (la - t->r0) + (lb - t->r0) * (lb - t->r0));
      double cth = (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / (la * lb);
      if (cth > 1.0) cth = 1.0;
      if (cth < -1.0) cth = -1.0;
      double th = acos(cth), sth = sqrt(1.0 - cth * cth);
      if (sth < 1e-12) sth = 1e-12;
      en += 0.5 * t->k_angle * (th - t->theta0) * (th - t->theta0);
      /* F_a = (k (th - th0) / sin th) * (b/(la lb) - cos th a/la^2), same for b */
      double g = t->k_angle * (th - t->theta0) / sth;
      for (int d = 0; d < 3; d++) {
        double f1 = fa * a[d] + g * (b[d] / (la * lb) - cth * a[d] / (la * la));
        double f2 = fb * b[d] + g * (a[d] / (la * lb) - cth * b[d] / (lb * lb));
        force[3 * (o + 1) + d] += f1;
        force[3 * (o + 2) + d] += f2;
        force[3 * o + d] -= f1 + f2;
      }
      e_at[o] += en;
    }
  } else {
    free(e_at);
    return ORC_ERR_INVALID_ARG;
  }
  double acc = 0.0;
  for (int64_t i = 0; i < n_atoms; i++) acc += e_at[i];
  *energy = acc;
  free(e_at);
  return ORC_OK;
}

/* Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw (SC 2011):
 * a round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
 * (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)) with
 * M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key grows by the Weyl increments
 * (0x9E3779B9, 0xBB67AE85) after each of the ten rounds. */
void orc_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {counter[0], counter[1], counter[2], counter[3]};
  uint32_t k[2] = {key[0], key[1]};
  const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  for (int round = 0; round < 10; round++) {
    uint64_t prod0 = M0 * (uint64_t)c[0];
    uint64_t prod1 = M1 * (uint64_t)c[2];
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c[1] ^ k[0];
    uint32_t n1 = (uint32_t)(prod1 & 0xffffffffu);
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c[3] ^ k[1];
    uint32_t n3 = (uint32_t)(prod0 & 0xffffffffu);
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    k[0] = k[0] + 0x9E3779B9u;
    k[1] = k[1] + 0xBB67AE85u;
  }
  for (int i = 0; i < 4; i++) out[i] = c[i];
}

/* The thermostat's three standard normals of atom a at step `step`, end
 * `half` of the step: Philox with counter {a, low and high words of step,
 * half} and key {low, high word of the seed}; the four words become
 * uniforms (w + 1/2) / 2^32 in (0, 1); Box-Muller (Box and Muller 1958):
 * z = sqrt(-2 ln u) (cos, sin)(2 pi v) for (u, v) = (u0, u1) gives the x and
 * y normals, the cosine branch of (u2, u3) the z normal. */
void orc_thermo_normals(uint64_t seed, int64_t a, int64_t step, int half, double z[3]) {
  const uint32_t ctr[4] = {(uint32_t)a, (uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32),
                           (uint32_t)half};
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  double u[4];
  for (int i = 0; i < 4; i++) u[i] = ((double)w[i] + 0.5) / 4294967296.0;
  const double two_pi = 2.0 * 3.14159265358979323846;
  z[0] = sqrt(-2.0 * log(u[0])) * cos(two_pi * u[1]);
  z[1] = sqrt(-2.0 * log(u[0])) * sin(two_pi * u[1]);
  z[2] = sqrt(-2.0 * log(u[2])) * cos(two_pi * u[3]);
}

int orc_set_thermostat(orc_state* s, double gamma, double kt, uint64_t seed) {
  if (!s || !(gamma >= 0.0) || !(kt >= 0.0) || !isfinite(gamma) || !isfinite(kt)) return ORC_ERR_INVALID_ARG;
  s->th_gamma = gamma;
  s->th_kt = kt;
  s->th_seed = seed;
  s->th_step = 0;
  return ORC_OK;
}

/* The O part of the OVRVO splitting (Sivak, Chodera and Crooks 2014): an
 * exact Ornstein-Uhlenbeck update of the velocities over dt/2,
 * v <- c v + sqrt(1 - c^2) sqrt(kT / m') z with c = exp(-gamma dt / 2) and
 * m' the mass in the units where the kinetic energy is m' v^2 / 2. */
static void orc_thermo_half(const orc_state* s, double* vel, const double* mass, const orc_mdterms* t, double dt,
                            int half) {
  const double c = exp(-0.5 * s->th_gamma * dt);
  const double sc = sqrt(1.0 - c * c);
  for (int64_t a = 0; a < s->n; a++) {
    double z[3];
    orc_thermo_normals(s->th_seed, a, s->th_step, half, z);
    const double sd = sqrt(s->th_kt / (mass[a] * t->mv2_to_energy));
    for (int d = 0; d < 3; d++) vel[3 * a + d] = c * vel[3 * a + d] + sc * sd * z[d];
  }
}

/* Velocity Verlet for the particles (Theory, numerical integration; the
 * mesh potential follows the Verlet/constraint update inside each compute),
 * within the OVRVO scheme when a thermostat is set. */
int orc_md_run(orc_state* s, double* pos, double* vel, const double* mass, const orc_mdterms* t,
               double dt, int32_t n_steps, double* energy_log, int32_t* cycles_log) {
  if (!s || !pos || !vel || !mass || !t || n_steps < 0) return ORC_ERR_INVALID_ARG;
  size_t n3a = 3 * (size_t)s->n;
  double* f = (double*)malloc(sizeof(double) * n3a);
  double* fo = (double*)malloc(sizeof(double) * n3a);
  if (!f || !fo) { free(f); free(fo); return ORC_ERR_OUT_OF_MEMORY; }
  double e4[4], eo;
  int worst = ORC_OK;
  int rc = orc_compute(s, pos, f, e4);
  if (rc < 0) { free(f); free(fo); return rc; }
  rc = orc_nonelectrostatic(t, s->n, pos, s->P.box, s->P.r_cut, fo, &eo);
  if (rc < 0) { free(f); free(fo); return rc; }
  for (size_t k = 0; k < n3a; k++) f[k] += fo[k];
  for (int32_t step = 0; step < n_steps; step++) {
    if (s->th_gamma > 0.0) orc_thermo_half(s, vel, mass, t, dt, 0);
    for (int64_t a = 0; a < s->n; a++)
      for (int d = 0; d < 3; d++) {
        vel[3 * a + d] += 0.5 * dt * f[3 * a + d] / mass[a] * t->force_to_acc;
        pos[3 * a + d] += dt * vel[3 * a + d];
      }
    rc = orc_compute(s, pos, f, e4);
    if (rc < 0) { free(f); free(fo); return rc; }
    if (rc > worst) worst = rc;
    rc = orc_nonelectrostatic(t, s->n, pos, s->P.box, s->P.r_cut, fo, &eo);
    if (rc < 0) { free(f); free(fo); return rc; }
    for (size_t k = 0; k < n3a; k++) f[k] += fo[k];
    for (int64_t a = 0; a < s->n; a++)
      for (int d = 0; d < 3; d++) vel[3 * a + d] += 0.5 * dt * f[3 * a + d] / mass[a] * t->force_to_acc;
    if (s->th_gamma > 0.0) orc_thermo_half(s, vel, mass, t, dt, 1);
    s->th_step++;
    double ekin = 0.0;
    for (int64_t a = 0; a < s->n; a++)
      for (int d = 0; d < 3; d++) ekin += 0.5 * mass[a] * vel[3 * a + d] * vel[3 * a + d] * t->mv2_to_energy;
    if (energy_log) {
      double* L = energy_log + 6 * (size_t)step;
      L[0] = e4[0]; L[1] = e4[1]; L[2] = e4[2]; L[3] = eo; L[4] = ekin;
      L[5] = e4[3] + eo + ekin;
    }
    if (cycles_log) cycles_log[step] = s->st.cycles;
  }
  free(f); free(fo);
  return worst;
}

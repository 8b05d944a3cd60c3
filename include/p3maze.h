/*
 * p3maze.h -- C ABI of the MI355X (gfx950) P3MaZe long-range electrostatics step.
 *
 * The problem is the one stated in the paper's Theory section: point charges
 * Q_b at positions r_b in a cubic periodic box of edge L, a Gaussian
 * screening of width sigma (Eq. 4) that splits the Coulomb energy into a
 * short-range pair sum, a smooth long-range mesh part and a self term
 * (Eqs. 5-7), a real-space cutoff R_c (Eq. 6), a cubic mesh of spacing
 * h = L/N carrying the potential of the smooth charges (Eq. 10), and a
 * B-spline assignment/interpolation order.  Each compute call is one step of
 * the constrained ("Mass-Zero") dynamics of the mesh potential: Verlet
 * prediction, correction problem M y = sigma_p (Eqs. 16-17) solved by
 * multigrid V-cycles to a max-norm residual tolerance (Eq. 26), field update
 * (Supporting Information, numerical integration), forces by interpolating a
 * central-difference mesh gradient (Eq. 21) plus the screened pair forces
 * (Eq. 20).
 *
 * Conventions shared by every entry point:
 *   - Return value: p3mz_status.  Negative = error, outputs undefined; the
 *     message is available from p3mz_last_error() (per thread).  Positive =
 *     warning, outputs valid.  No C++ exception crosses this boundary.
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *     tensors' data_ptr) on the device the context was created on;
 *     *_host are host pointers.  The caller owns them; the library never
 *     frees or keeps them beyond the call.
 *   - stream: a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it; a call returns after enqueueing, except where
 *     a comment says it synchronises.
 *   - Particle arrays are array-of-structures [n][3] doubles; positions may
 *     be in any periodic image.  Mesh arrays are [N][N][N] doubles with x
 *     fastest.
 *   - Units are the caller's: lengths as the box, charges as given, energies
 *     and forces scaled by coulomb_k.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef P3MAZE_H
#define P3MAZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  P3MZ_OK = 0,
  P3MZ_WARN_NOT_CONVERGED = 1,   /* cycle cap reached; results written, stats hold the residual */
  P3MZ_ERR_INVALID_ARG = -1,     /* NULL pointer, parameter out of range, r_cut > L/2 ... */
  P3MZ_ERR_NOT_NEUTRAL = -2,     /* |sum Q| > 1e-10 sum |Q|: the periodic problem has no solution */
  P3MZ_ERR_MESH_SHAPE = -3,      /* N not 4*2^m (m >= 1), or h too coarse for sigma */
  P3MZ_ERR_OUT_OF_MEMORY = -4,
  P3MZ_ERR_HIP = -5,             /* a HIP runtime call failed */
  P3MZ_ERR_NAN = -6,             /* non-finite position */
  P3MZ_ERR_STATE = -7,           /* call not valid in the context's state (e.g. bad state blob) */
  P3MZ_ERR_DENSITY = -8          /* too many atoms in one spatial bin for the deterministic sort */
} p3mz_status;

/* FP64: every stage in FP64.  MIXED: the V-cycle and the gather in FP32,
 * the charge source, sigma_p, the outer residual, projections, coarsest
 * solve and updates in FP64.  MIXED32: as MIXED with an FP32 charge
 * source: the assigned charges (summed in FP64) are stored and smoothed in
 * FP32; sigma_p is still formed in FP64 from the widened FP32 charges.  The
 * rounding noise (~1e-7 of max|q^s|, new every step and amplified by the
 * multiplier extrapolation) perturbs the residual sequence; at tolerances
 * of 1e-6 and above the V-cycle counts match an FP64 reference, at 1e-8 it
 * costs extra V-cycles.  Meant for tol >= 1e-6. */
typedef enum { P3MZ_PREC_FP64 = 0, P3MZ_PREC_MIXED = 1, P3MZ_PREC_MIXED32 = 2 } p3mz_precision;

/* Control parameters of the problem statement (Theory; protocol paragraphs
 * of the molten-salt and water results). */
typedef struct {
  double box;          /* cubic edge L > 0                                             */
  double alpha;        /* Ewald splitting > 0; Gaussian width sigma = 1/(sqrt(2) alpha) */
  double r_cut;        /* real-space cutoff R_c, 0 < R_c <= L/2 (minimum image),
                          alpha * R_c <= 32                                            */
  int32_t mesh;        /* N points per edge, N = 4*2^m, 1 <= m <= 7 (8, 16, ..., 512)   */
  int32_t order;       /* B-spline order p, 2..7 (the paper uses cubic, p = 4)          */
  double tol;          /* residual tolerance > 0                                        */
  int32_t tol_mode;    /* 0: max|M y - sigma_p| <= tol * max|q^s|; 1: <= tol (absolute) */
  int32_t max_cycles;  /* V-cycle cap per step, 0..64                                   */
  int32_t predictor;   /* multiplier predictor: 0 (Verlet prediction only, the in-house
                          real-space P3M start), 1: y^k, 2: 2y^k - y^{k-1},
                          3: 3y^k - 3y^{k-1} + y^{k-2}                                  */
  int32_t precision;   /* p3mz_precision.  MIXED: V-cycle sweeps, restriction and
                          prolongation, and the force gather in FP32; charge
                          assignment, smoothing, sigma_p, the outer residual,
                          zero-mean projections, coarsest solve and the
                          multiplier/potential updates in FP64.  MIXED32:
                          assigned charges stored and smoothed in FP32 as
                          well (for tol >= 1e-6)                           */
  double coulomb_k;    /* Coulomb constant k_e (1 for Gaussian units)                   */
  int32_t nu_pre;      /* red-black Gauss-Seidel sweeps before restriction, >= 0;
                          -1: the autotuned or default (2) value                       */
  int32_t nu_post;     /* ... after prolongation; -1 as above; nu_pre+nu_post >= 1      */
  int32_t excl_group;  /* 0: no exclusions; g > 0: atoms i, j with i/g == j/g interact
                          only through the mesh minus its erf part (rigid-molecule
                          exclusion, e.g. g = 3 for O,H,H water)                      */
  int32_t stencil;     /* mesh discretisation.  0: the seven-point Laplacian M and the
                          two-point central gradient (second order; Eq. 10, Eq. 21).
                          1: fourth order, the Hermitian (Mehrstellen) form the paper
                          names after Eq. 21 as the higher-order option: the
                          constraint A phi = -(4 pi / h) B q^s with the 19-point
                          A = (1/6)(2 sum_faces + sum_edges - 24) and
                          B = (1/12)(sum_faces + 6), the four-point gradient
                          (8 (f+1 - f-1) - (f+2 - f-2)) / 12h, smoothing weight
                          nu <= 1/6; the V-cycles keep M (defect correction, more
                          cycles per step).  Needs order <= 5                         */
} p3mz_params;

typedef struct {
  int32_t status;            /* status of the last compute                            */
  int32_t cycles;            /* V-cycles of the last compute                          */
  int32_t cold;              /* 1 if the last compute was a cold solve               */
  int32_t m_eff;             /* predictor order actually used (ramped by history)    */
  int32_t nu_pre, nu_post;   /* resolved sweep counts                                 */
  int32_t K;                 /* smoothing steps per dimension                         */
  int32_t levels;            /* multigrid levels down to 4^3                          */
  double nu_smooth;          /* smoothing step weight                                 */
  double thresh;             /* residual threshold of the last compute               */
  double norm_qs;            /* max |q^s|                                             */
  double res_hist[65];       /* residual before cycle c, c = 0..cycles                */
  double e_sr, e_lr, e_self, e_total;
  int64_t steps;             /* completed compute calls since create/load            */
  int32_t graphs;            /* 1 if the last step ran from captured graphs         */
  /* with p3mz_set_timing on, milliseconds of the last step from HIP events on
   * the caller's stream: the mesh step (binning, spread, smoothing, constraint
   * solve, field update, gather) and the short-range pairs; the split of the
   * mesh step into spread+smoothing / solve+update / gather only when the
   * step was launched kernel by kernel (else -1). */
  double ms_mesh, ms_short_range, ms_spread, ms_solve, ms_gather;
  /* sum over all atoms of the electrostatic force (short range + mesh) the
   * last compute wrote: zero up to rounding for the pair part, and to the
   * solver tolerance for the mesh part (the central-difference gradient is
   * antisymmetric; Eq. 21 and the momentum paragraph after it).  NaN when
   * the call wrote no forces. */
  double net_force[3];
} p3mz_stats;

typedef struct p3mz_ctx p3mz_ctx;

/* Allocate a context for n_atoms charges (host array, copied).  Plans the
 * mesh hierarchy and allocates every workspace on the current HIP device, so
 * compute never allocates.  Errors: INVALID_ARG, MESH_SHAPE, NOT_NEUTRAL,
 * OUT_OF_MEMORY, HIP.  On error *out is NULL. */
p3mz_status p3mz_create(const p3mz_params* params, int64_t n_atoms, const double* charges_host,
                        p3mz_ctx** out);

/* One mesh step at positions pos_dev [n][3].  Writes force_dev [n][3]
 * (short-range + long-range electrostatic force, overwritten) and
 * energy_dev [4] = {E_sr, E_lr, E_self, E_total}.  The first call after
 * create/reset is a cold solve from a zero potential; later calls warm-start
 * from the stored potential and multiplier history.  Synchronises the stream
 * while deciding the number of V-cycles.  force_dev / energy_dev may be NULL
 * to skip those outputs (the mesh potential is still advanced).  Errors:
 * INVALID_ARG, NAN, DENSITY, HIP; warning NOT_CONVERGED. */
p3mz_status p3mz_compute(p3mz_ctx* ctx, const double* pos_dev, double* force_dev,
                         double* energy_dev, void* stream);

/* Copy an internal mesh of the last compute to phi_dev ([N][N][N] doubles,
 * x fastest): which = 0 assigned charges q, 1 smoothed q^s, 2 sigma_p
 * (zero-mean), 3 multiplier y, 4 potential phi^{k+1}, 5 previous potential.
 * FP32 meshes of the mixed mode are widened exactly. */
p3mz_status p3mz_get_mesh(p3mz_ctx* ctx, int32_t which, double* out_dev, void* stream);

/* The mesh potential phi^{k+1} of the last compute (the field the forces
 * were interpolated from; Eq. 21 and the field update of the Supporting
 * Information) into phi_dev ([N][N][N] doubles, x fastest, zero mean, the
 * potential of the smoothed charges in coulomb_k = 1 units).  Same as
 * p3mz_get_mesh(ctx, 4, ...).  Enqueued on stream.  Errors: INVALID_ARG. */
p3mz_status p3mz_get_potential(p3mz_ctx* ctx, double* phi_dev, void* stream);

/* One V-cycle of the context's schedule for M e = r on the finest mesh:
 * r_dev, e_dev [N][N][N] doubles (e is overwritten).  In mixed mode r is
 * rounded to FP32 and the cycle runs in the mixed precision of the step.
 * Leaves the potential history untouched. */
p3mz_status p3mz_vcycle(p3mz_ctx* ctx, const double* r_dev, double* e_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * V-cycle of p3mz_vcycle without a context.  One V-cycle with the schedule
 * (nu_pre, nu_post) for M e = r on an N^3 mesh, r_dev and e_dev [N][N][N]
 * doubles (x fastest, e overwritten; mixed precision rounds r to FP32 and
 * runs the cycle in the mixed precision of a step).  The result equals
 * p3mz_vcycle of a context with the same mesh, precision and schedule.
 * The level hierarchy, the coarsest-level Green's function and the control
 * block live in a fixed device array of 8 MiB per GPU, held until the
 * process ends, so N <= 64.  The call allocates nothing; its first call on
 * a device locates that device's array and synchronises the device.  All
 * calls on one GPU share the array: calls that overlap in time on one GPU
 * (other streams, other threads) race.  Errors: INVALID_ARG for NULL
 * pointers, N not 4*2^m in 8..64, a bad precision or schedule; HIP. */
p3mz_status p3mz_vcycle_noalloc(int32_t mesh, int32_t precision, int32_t nu_pre, int32_t nu_post,
                                const double* r_dev, double* e_dev, void* stream);

/* Statistics of the last compute (host struct). */
p3mz_status p3mz_get_stats(const p3mz_ctx* ctx, p3mz_stats* out);

/* Forget the potential/multiplier history: the next compute is a cold solve. */
p3mz_status p3mz_reset_history(p3mz_ctx* ctx);

/* Serialise the history {phi^k, phi^{k-1}, stored multipliers, counters} into
 * host_buf.  With host_buf == NULL, *bytes receives the size.  Synchronises. */
p3mz_status p3mz_save_state(const p3mz_ctx* ctx, void* host_buf, size_t* bytes);
/* Restore a blob written by p3mz_save_state of a context with the same mesh
 * and precision.  Errors: STATE if the blob does not match. */
p3mz_status p3mz_load_state(p3mz_ctx* ctx, const void* host_buf, size_t bytes);

/* Non-electrostatic terms for p3mz_md_run (eV / Angstrom / amu / fs style
 * units are the caller's choice, fixed by the two conversion factors). */
typedef struct {
  int32_t model;        /* 0 none, 1 stand-in Born-Mayer repulsion between all pairs,
                           2 flexible three-site water (atoms O,H,H per molecule)   */
  double bm_a, bm_rho;  /* model 1: A exp(-r/rho), shifted to zero at r_cut         */
  double lj_eps, lj_sigma;   /* model 2: O-O Lennard-Jones, shifted to zero at r_cut */
  double k_bond, r0;    /* model 2: 0.5 k (r - r0)^2 per O-H bond                   */
  double k_angle, theta0;    /* model 2: 0.5 k (theta - theta0)^2, radians          */
  double force_to_acc;  /* acceleration = force / mass * force_to_acc              */
  double mv2_to_energy; /* kinetic energy = 0.5 m v^2 * mv2_to_energy               */
} p3mz_mdterms;

/* n_steps of velocity Verlet (Theory, numerical integration) driving one
 * mesh step per MD step.  pos_dev/vel_dev [n][3] are advanced in place;
 * mass_dev [n].  energy_log_dev [n_steps][6] = {E_sr, E_lr, E_self,
 * E_other, E_kin, E_total}; cycles_log_dev [n_steps] V-cycles per step
 * (either may be NULL).  The first call computes the forces at the initial
 * positions before the first step (a cold solve on first use); a later call
 * continues the trajectory from the forces the last one left, provided it
 * passes the same pos/vel/mass buffers and terms and nothing else (a
 * p3mz_compute, a state load or reset) ran in between; otherwise it
 * recomputes the forces at the given positions first.  Synchronises once
 * per step.  Errors as p3mz_compute. */
p3mz_status p3mz_md_run(p3mz_ctx* ctx, double* pos_dev, double* vel_dev, const double* mass_dev,
                        const p3mz_mdterms* terms, double dt, int32_t n_steps,
                        double* energy_log_dev, int32_t* cycles_log_dev, void* stream);

/* Langevin thermostat for p3mz_md_run, in the OVRVO splitting: each step
 * starts with v <- a v + b sqrt(kT / (m * mv2_to_energy)) z (a = exp(-gamma
 * dt / 2), b = sqrt(1 - a^2), z independent standard normals per component),
 * then the half kick, the drift, the forces and the half kick, and ends with
 * the same velocity update with new normals (Sivak, Chodera and Crooks' OVRVO
 * scheme, the Langevin integrator of the paper's equilibration runs).  gamma
 * is the friction in inverse time units of dt (0: no thermostat, plain
 * velocity Verlet, the default); kT in energy units.  The normals come from
 * Philox4x32-10 with key = seed and counter {atom, step (64 bits), end of the
 * step (0, 1)}, uniforms (x + 1/2) 2^-32, then Box-Muller: (x0, x1) give the
 * x and y normals, (x2, x3) the z normal.  The step counter restarts at 0 with
 * every call; batched MD runs without a thermostat.  Synchronises the device.
 * Errors: INVALID_ARG for negative or non-finite gamma or kT. */
p3mz_status p3mz_set_thermostat(p3mz_ctx* ctx, double gamma, double kT, uint64_t seed);

/* Launch mode.  By default (on = 1) each step is enqueued as three captured
 * HIP graphs -- before the solve, one V-cycle (replayed once per cycle), after
 * the solve -- captured on a private stream at first use and re-captured only
 * when the caller's buffer pointers change; on = 0 launches every kernel
 * directly.  Results are bitwise identical.  Synchronises the device. */
p3mz_status p3mz_set_graphs(p3mz_ctx* ctx, int32_t on);

/* Record HIP events between the stages of every compute (on = 1) so that
 * p3mz_stats.ms_stage holds their durations; on = 0 stops it.  Costs five
 * event records per compute. */
p3mz_status p3mz_set_timing(p3mz_ctx* ctx, int32_t on);

/* Kernel families on the finest mesh level that can be timed launch by
 * launch with HIP events on the compute stream. */
enum {
  P3MZ_KERNEL_HALFSWEEP = 0,  /* red or black Gauss-Seidel half-sweep             */
  P3MZ_KERNEL_OUTER = 1,      /* FP64 outer residual + multiplier update          */
  P3MZ_KERNEL_SMOOTH = 2,     /* one axis of the charge smoothing                 */
  P3MZ_KERNEL_RESTRICT = 3,   /* fused residual + full-weighting restriction      */
  P3MZ_KERNEL_PROLONG = 4,    /* trilinear correction of the black points         */
  P3MZ_KERNEL_SWEEP0 = 5,     /* first sweep from a zero correction               */
  P3MZ_KERNEL_TAIL = 6,       /* one-workgroup coarse levels (<= 16^3; 32^3 in batches) + 4^3 solve */
  P3MZ_KERNEL_SPREAD = 7, P3MZ_KERNEL_GATHER = 8, P3MZ_KERNEL_SR = 9,
  P3MZ_KERNEL_SIGMA = 10, P3MZ_KERNEL_PHI = 11,
  P3MZ_KERNEL_FUSED_DOWN = 12, /* fused down leg of a small level (first sweep + pairs) */
  P3MZ_KERNEL_FUSED_UP = 13,  /* fused up leg of a small level (correction + pairs)    */
  /* batches only: `reps` finest-level half-sweeps of every system in ONE
   * persistent launch (workgroups take (sweep, system, tile) tasks from a
   * device counter; a system's next sweep waits on a per-system device
   * barrier), timed per half-sweep against HALFSWEEP's one launch per sweep */
  P3MZ_KERNEL_PERSIST_HALFSWEEP = 14
};
/* Start timing one kernel family (kernel_id as above, -1 = off) and zero the
 * totals.  Up to 2048 launches per compute are timed.  While a family is timed
 * the step is launched kernel by kernel (no graphs). */
p3mz_status p3mz_set_kernel_timer(p3mz_ctx* ctx, int32_t kernel_id);
/* Totals since p3mz_set_kernel_timer: summed event milliseconds, number of
 * timed launches and the summed algorithmic HBM bytes of those launches
 * (the bytes the method must move per launch, independent of caching). */
p3mz_status p3mz_get_kernel_timer(const p3mz_ctx* ctx, double* total_ms, int64_t* launches,
                                  double* total_bytes);
/* The same launches one by one, in launch order: ms_host[i] (event
 * milliseconds) and bytes_host[i] (algorithmic bytes) for the first
 * min(max, launches) of them (up to 65536 are kept); *count = the number
 * written.  Launches that found the solve already converged return at once
 * and show as short durations.  Errors: INVALID_ARG for NULL pointers. */
p3mz_status p3mz_get_kernel_launches(const p3mz_ctx* ctx, int32_t max, float* ms_host, double* bytes_host,
                                     int32_t* count);

/* Back-to-back timing of one finest-level kernel on the context's current
 * buffers: `reps` launches between two HIP events on `stream`; *avg_ms is the
 * mean launch duration and *bytes_per_launch its algorithmic HBM traffic.
 * Families: HALFSWEEP, SWEEP0, RESTRICT, PROLONG, TAIL, FUSED_DOWN and
 * FUSED_UP (finest level fused), SMOOTH (x axis),
 * OUTER and SIGMA (without their one-workgroup finalize pass), SPREAD and
 * GATHER (on the last step's binning, no forces written).  Overwrites
 * scratch buffers only; the potential and multiplier history is untouched.
 * Synchronises the stream.  Errors: INVALID_ARG for other families or a mesh
 * without that kernel. */
p3mz_status p3mz_kernel_bench(p3mz_ctx* ctx, int32_t kernel_id, int32_t reps, void* stream, double* avg_ms,
                              double* bytes_per_launch);

/* Set the V-cycle schedule (red-black sweeps before restriction and after
 * prolongation, 0..16 each, sum >= 1) and the smoothing launch shape
 * (0 .. P3MZ_SMOOTH_TILES-1, shapes that divide the mesh edge; all shapes give
 * identical results).  Synchronises the device; graphs are recaptured. */
#define P3MZ_SMOOTH_TILES 7
p3mz_status p3mz_set_schedule(p3mz_ctx* ctx, int32_t nu_pre, int32_t nu_post, int32_t smooth_tile);

/* Multigrid levels above the one-workgroup tail whose edge is at most
 * max_edge (the 32^3 and 64^3 levels qualify; 0 = none) run each leg of the
 * V-cycle (the pre-smoothing sweeps, and the correction plus post-smoothing
 * sweeps) as one launch: each workgroup keeps a tile of grid rows with a halo
 * of one row per sweep in LDS and recomputes the halo instead of exchanging
 * it (temporal blocking).  The down leg also forms the restricted residual of
 * its tile when a box two rows wider fits.  Needs nu_pre, nu_post >= 1 and
 * the halo box within 160 KiB of LDS; other levels and schedules keep one
 * launch per sweep.  Results are bitwise identical either way.  Default 64;
 * systems of a batch always keep one launch per sweep.  Synchronises the
 * device; graphs are recaptured.  Errors: INVALID_ARG for max_edge < 0. */
p3mz_status p3mz_set_fused_levels(p3mz_ctx* ctx, int32_t max_edge);

/* Short-range pair sums (Eq. (6) with the exclusion correction of Eq. (20),
 * and the MD pair terms) over Verlet neighbour lists with a skin: each list
 * holds every atom within r_cut + skin at its build; a build is triggered on
 * the device when some atom has moved more than skin/2 (minimum image) since
 * the last one, so every pair within r_cut is always in the lists and the
 * results equal those of a fresh cell scan up to summation order.  The cell
 * list is then made of cells at least r_cut + skin wide.  skin in [0, r_cut]
 * (0: no lists, the cells are scanned every step); capacity = entries per
 * atom, 0 for 30 % above the count expected at the mean density plus 64
 * (rounded up to 64; an atom with more neighbours falls back to the cell
 * scan).  The lists take n_atoms * capacity * 4 bytes of device memory.
 * Default: skin 0.1 r_cut, automatic capacity; systems of a batch scan the
 * cells.  Synchronises the device; graphs are recaptured; the next step
 * builds the lists.  Errors: INVALID_ARG for skin outside [0, r_cut] or
 * capacity < 0 (the lists stay as they were); OUT_OF_MEMORY or HIP (the
 * context is left without lists, scanning the cells). */
p3mz_status p3mz_set_neighbor_list(p3mz_ctx* ctx, double skin, int32_t capacity);

/* Neighbour-list builds so far, atoms found over capacity summed over those
 * builds, and the capacity (0: no lists), as of the last completed step. */
p3mz_status p3mz_get_neighbor_stats(const p3mz_ctx* ctx, int64_t* builds, int64_t* over_capacity,
                                    int32_t* capacity);

typedef struct {
  int32_t nu_pre, nu_post;   /* chosen schedule                                        */
  int32_t smooth_tile;       /* chosen smoothing launch shape                          */
  int32_t n_candidates;      /* schedules tried                                        */
  double ms_best;            /* mean mesh-step milliseconds per frame, chosen schedule */
  double ms_default;         /* the same for the default (2, 2)                        */
  double ms_smooth;          /* three smoothing passes with the chosen shape           */
  int32_t cand_nu_pre[16], cand_nu_post[16], cand_cycles[16];
  double cand_ms[16];         /* mean measured mesh-step milliseconds per frame          */
  double cand_ms_cycle[16];   /* milliseconds of one V-cycle plus the outer residual      */
  double cand_cycles_frac[16];   /* mean fractional cycle count (residual interpolated)   */
  double cand_expected_ms[16];   /* the criterion: cand_ms corrected to the expected count */
} p3mz_tune_result;

/* Autotuner.  Times the smoothing launch shapes back to back, then every
 * candidate V-cycle schedule by time to tolerance: each candidate restarts
 * from the context's current history and runs mesh steps on the caller's
 * frames_dev [n_frames][n_atoms][3] (1 <= n_frames <= 64, e.g. the next
 * positions of a trajectory).  A step's cycle count is its fractional count
 * X (where the residual, interpolated geometrically within the last cycle,
 * crosses the threshold) rounded up, so over a trajectory it averages about
 * mean X + 1/2; the measured mean mesh-step time is corrected to that count
 * with the candidate's time per cycle (one V-cycle and the outer residual),
 * and the schedule with the least corrected time wins.  The context is left with its history unchanged and
 * the chosen schedule applied; the choice is stored in the tuning cache
 * (JSON; path from the environment variable P3MZ_TUNE_CACHE, default
 * $HOME/.cache/p3maze/tune.json) under (device, mesh, order, precision),
 * where contexts created with nu_pre or nu_post = -1 find it.  Results of a
 * step depend on the schedule (cycle counts differ); a reference run must
 * use the same schedule (p3mz_stats.nu_pre/nu_post).  Errors: INVALID_ARG
 * when the cache cannot be written. */
p3mz_status p3mz_autotune(p3mz_ctx* ctx, const double* frames_dev, int32_t n_frames, void* stream,
                          p3mz_tune_result* out);

void p3mz_destroy(p3mz_ctx* ctx);

/* ---- Batched replicas ------------------------------------------------------
 * Many independent systems (uneven atom counts and meshes) advanced together:
 * every kernel of the step is launched once for all systems, with one
 * workgroup row per system, so small systems share the GPU instead of
 * leaving it idle.  Each system runs exactly the algorithm of a single
 * context with its own parameters and history (same results, bitwise), and
 * converges on its own: the V-cycle launches of a system that has met its
 * tolerance return at once.  All systems of a batch need the same precision.
 *
 * Packed layout: system s owns atoms [off_s, off_s + n_atoms[s]) of every
 * packed per-atom array, off_s = sum of the earlier n_atoms; positions,
 * forces and velocities are [atom][3] FP64, masses [atom].  The caller owns
 * every device pointer; launches are recorded (and captured as HIP graphs)
 * against the pointers of the first call and recorded again when they
 * change. */
typedef struct p3mz_batch p3mz_batch;

/* per_sys[n_sys] parameters and n_atoms[n_sys] atom counts; host charges,
 * packed.  Each system is validated as by p3mz_create (same errors); all
 * device memory is allocated here.  Errors: INVALID_ARG when precisions
 * differ. */
p3mz_status p3mz_batch_create(int32_t n_sys, const p3mz_params* per_sys, const int64_t* n_atoms,
                              const double* charges_packed_host, p3mz_batch** out);
/* One mesh step (as p3mz_compute) for every system: pos_dev packed, read
 * only; force_dev packed (SR+LR, overwritten); energies_dev [n_sys][4] =
 * {E_sr, E_lr, E_self, E_total} per system.  Per-system statistics via
 * p3mz_batch_get_stats.  WARN_NOT_CONVERGED if any system hit its cycle cap;
 * NAN if any system saw a non-finite position (that system's history is
 * dropped).  Synchronises once per V-cycle batch. */
p3mz_status p3mz_batch_compute(p3mz_batch* b, const double* pos_dev, double* force_dev, double* energies_dev,
                               void* stream);
/* n_steps of velocity Verlet for every system (as p3mz_md_run, one MD step
 * of all systems per iteration).  energy_log_dev [n_sys][n_steps][6] and
 * cycles_log_dev [n_sys][n_steps] (either may be NULL). */
p3mz_status p3mz_batch_md_run(p3mz_batch* b, double* pos_dev, double* vel_dev, const double* mass_dev,
                              const p3mz_mdterms* terms, double dt, int32_t n_steps, double* energy_log_dev,
                              int32_t* cycles_log_dev, void* stream);
/* One velocity-Verlet MD step of every system (p3mz_batch_md_run with
 * n_steps = 1), returning what the step computed: force_dev packed [atom][3]
 * (the total force the closing half kick used: electrostatic plus the
 * non-electrostatic terms), energies_dev [n_sys][4] = {E_sr, E_lr, E_self,
 * E_total} (electrostatic) and cycles_dev [n_sys] V-cycles of the step's
 * solve; each of the three may be NULL.  Errors as p3mz_batch_md_run. */
p3mz_status p3mz_batch_step(p3mz_batch* b, double* pos_dev, double* vel_dev, const double* mass_dev,
                            const p3mz_mdterms* terms, double dt, double* force_dev, double* energies_dev,
                            int32_t* cycles_dev, void* stream);
/* Statistics of system `sys` after the last batched step. */
p3mz_status p3mz_batch_get_stats(const p3mz_batch* b, int32_t sys, p3mz_stats* out);
/* Events around the mesh part (spread .. gather) and the pair part of every
 * batched step (on = 1); p3mz_batch_get_timing returns the last step's
 * milliseconds and whether it ran from captured graphs. */
p3mz_status p3mz_batch_set_timing(p3mz_batch* b, int32_t on);
p3mz_status p3mz_batch_get_timing(const p3mz_batch* b, double* ms_mesh, double* ms_short_range, int32_t* graphs);
/* Captured graphs (default) or direct launches; results are identical. */
p3mz_status p3mz_batch_set_graphs(p3mz_batch* b, int32_t on);
/* As p3mz_kernel_bench, for one batched launch of a V-cycle kernel family
 * (HALFSWEEP, SWEEP0, RESTRICT, PROLONG, TAIL) over every system's finest
 * level; *bytes_per_launch sums the systems' algorithmic bytes.  With
 * PERSIST_HALFSWEEP, one persistent launch runs `reps` half-sweeps and
 * *avg_ms is its time per half-sweep (STATE if a device wait gave up).
 * Leaves each system's control block open (the next step resets it). */
p3mz_status p3mz_batch_kernel_bench(p3mz_batch* b, int32_t kernel_id, int32_t reps, void* stream, double* avg_ms,
                                    double* bytes_per_launch);
void p3mz_batch_destroy(p3mz_batch* b);
const char* p3mz_status_string(p3mz_status s);
const char* p3mz_last_error(void);
/* Library version string, e.g. "p3maze-gfx950 0.1". */
const char* p3mz_version(void);

#ifdef __cplusplus
}
#endif
#endif

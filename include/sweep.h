/*
 * sweep.h -- C ABI of the MI355X (gfx950) transport-sweep library.
 *
 * The library solves the discrete-ordinates form of the steady radiative
 * transfer equation with isotropic scattering (Peter et al. 2022, "The Sweep
 * Method for radiative Transfer in Arepo", eq. radiativeTransfer of sec. 2.2)
 * on Voronoi grids by transport sweeps (sec. 2.3-2.5):
 *
 *   - a task is a (cell, direction) pair and is solved for all frequency groups
 *     at once (sec. 2.5);
 *   - for direction Omega the half-face f of cell c with unit normal n_f
 *     (outward, n = (p'-p)/|p'-p| on Voronoi grids, appendix A) is an outflow
 *     face if s = Omega.n_f > eps_tie, an inflow face if s < -eps_tie, and
 *     carries nothing otherwise; its weight is w = A_f |s|;
 *   - the inflow faces with an interior (non-periodic) neighbour define the
 *     per-direction dependency graph, acyclic on Voronoi grids (appendix A);
 *   - each task solves the first-order upwind balance of transport scheme (a)
 *     (sec. 2.6): the cell's outflow is split over its outflow faces in
 *     proportion to A_i (n_i . Omega), so with Aperp = sum of outflow w
 *        (Aperp + kappa V) phi = sum_{inflow f} w_f phi_upwind(f) + S,
 *     S = L/D + kappa_s V sum_d' phi_prev(d') / D  (source iteration, alg. 1);
 *   - periodic faces (non-zero image shift) are cut from the graph; what leaves
 *     through them re-enters the partner cell in the next pass (sec. 2.7).
 *
 * phi is the intensity integrated over the direction's solid angle 4 pi / D
 * (photons/s per unit area).  Outputs per cell and group:
 *   J = (1/4pi) sum_d phi          absorbed = kappa_a V sum_d phi
 * with kappa_a = (1 - albedo) kappa, kappa being the extinction coefficient.
 *
 * Exponential cell law (opts->law = SWEEP_LAW_EXP): the attenuation form
 * 1 - e^{-dn sigma} of the paper's scattering test (sec. 3.3), with the mean
 * distance travelled in the cell taken as the mean chord V / Aperp, so the
 * optical depth of a task is tau = kappa V / Aperp.  The power entering the
 * task, T = sum_{inflow f} w_f x_upwind(f) + S, leaves with the factor e^{-tau}
 * through the outflow faces (exit flux density x = T e^{-tau} / Aperp, what the
 * downwind cells, the walls and the periodic partners receive per unit w) and
 * T (1 - e^{-tau}) is absorbed; the cell average that enters J, absorbed and
 * the scattering source is phi = T (1 - e^{-tau}) / (kappa V) (T / Aperp at
 * kappa = 0).  tau is capped at 40 for the transmission (a thicker cell passes
 * on e^{-40} = 4.2e-18 of T), which keeps x in the normal FP32 range so that
 * phi can be recovered from it.  Requires Aperp > 0 (every closed cell).
 *
 * Conventions for every call:
 *   - every function returns sweep_status_t; on failure sweep_last_error()
 *     returns a thread-local message; no exception or abort crosses the ABI;
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory;
 *   - per-cell-per-group arrays are cell-major with the G groups contiguous
 *     ([C_total][G], row-major), cells of all meshes concatenated in mesh
 *     order (global cell id = mesh offset + local id);
 *   - work is enqueued on the caller's `stream` (a hipStream_t, NULL = null
 *     stream); only sweep_build_dag, sweep_dag_export, sweep_dag_level_widths,
 *     sweep_tune, sweep_ion_step, sweep_ion_step_noalloc, sweep_sync, and
 *     sweep_forward / sweep_adjoint with pbc_tol or check set synchronise
 *     that stream;
 *   - inputs that only the kernels see (kappa and emission negative or not
 *     finite, a task whose denominator Aperp + kappa V is not positive, loss
 *     gradients that are not finite) raise an error flag kept with the DAG;
 *     the next call on that DAG that synchronises (sweep_sync, sweep_dag_export,
 *     sweep_tune, sweep_ion_step(_noalloc), pbc_tol or check) returns
 *     SWEEP_ERR_INVALID_ARG for it and clears it.  The outputs of the call that
 *     saw such input are not meaningful;
 *   - the caller owns every array argument and output; outputs are fully
 *     overwritten; the library owns the DAG object and its internal buffers.
 */
#ifndef SWEEP_H_
#define SWEEP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SWEEP_OK = 0,
  SWEEP_ERR_INVALID_ARG = -1, /* bad argument or malformed mesh */
  SWEEP_ERR_CYCLE = -2,       /* a dependency graph is cyclic (no topological order) */
  SWEEP_ERR_OOM = -3,         /* device allocation failed */
  SWEEP_ERR_HIP = -4,         /* a HIP runtime call failed */
  SWEEP_ERR_NOT_BUILT = -5,   /* NULL or destroyed DAG handle */
  SWEEP_ERR_UNSUPPORTED = -6  /* valid request that this library does not implement */
} sweep_status_t;

/* Number of FP64 totals per (mesh, group), see sweep_forward. */
#define SWEEP_N_TOTALS 8

/* One Voronoi grid.  All pointers are DEVICE pointers and must stay valid
 * for the duration of sweep_build_dag only (the DAG keeps what it needs). */
typedef struct {
  int32_t n_cells;
  int64_t n_half_faces;
  const int64_t* face_ptr;    /* [n_cells+1] CSR offsets of each cell's half-faces */
  const int32_t* face_nbr;    /* [n_half_faces] neighbour cell (local id), -1 = vacuum wall */
  const int32_t* face_twin;   /* [n_half_faces] matching half-face of the neighbour, -1 for
                                 walls; used only by validation, may be NULL */
  const int8_t* face_shift;   /* [n_half_faces] periodic image code, 0 = none; NULL = no
                                 periodic faces */
  const double* face_area;    /* [n_half_faces] */
  const double* face_normal;  /* [3*n_half_faces] unit normal, outward from the owner */
  const double* cell_volume;  /* [n_cells] */
} sweep_mesh_t;

/* Transport schemes of sec. 2.6: how a cell's outflow Aperp phi is shared among
 * its outflow faces (see sweep_build_opts_t.scheme). */
enum { SWEEP_SCHEME_AREA = 0, SWEEP_SCHEME_ALIGNED = 1 };

typedef struct {
  double eps_tie;   /* |Omega.n| <= eps_tie: the face carries nothing (default 1e-12) */
  int32_t validate; /* 1: check the mesh and directions on the host first (default 1) */
  int32_t kahn_counters; /* where the level computation keeps its per-cell dependency
                            counters: 0 = LDS when the largest mesh fits (4 bits per
                            cell), else global memory; 1 = LDS (UNSUPPORTED if the mesh
                            does not fit); 2 = global memory.  The levels do not depend
                            on it */
  int32_t scheme;   /* SWEEP_SCHEME_AREA (default): scheme (a), each outflow face i gets
                       the share A_i (n_i . Omega) / Aperp (weight w = A |s|).
                       SWEEP_SCHEME_ALIGNED: scheme (b), direction-conserving transport:
                       the n outflow faces with the largest Omega . n (ties: the lower
                       face index) each carry Aperp / n and the others nothing, so a
                       task has at most n downwind dependencies; needs every mesh's
                       face_twin.  The graph, the sweeps, the periodic passes and the
                       adjoint all follow the chosen scheme */
  int32_t n_aligned; /* scheme (b): n, 1..4 (0 = 3, the number of dimensions) */
  int32_t reserved[4];
} sweep_build_opts_t;

/* Opaque handle of a built set of per-direction dependency graphs. */
typedef struct sweep_dag_s* sweep_dag_t;

typedef struct {
  int32_t n_meshes;
  int32_t n_dirs;
  int64_t n_cells;        /* all meshes */
  int64_t n_tasks;        /* n_cells * n_dirs */
  int64_t n_up_entries;   /* upwind-row entries: graph edges seen from the downwind side */
  int64_t n_down_entries; /* graph edges seen from the upwind side */
  int32_t max_depth;      /* longest critical path (levels) over all (mesh, direction) */
  int32_t min_depth;
  double mean_depth;
  int64_t device_bytes;   /* bytes held by the DAG */
  int32_t kahn_lds_counters; /* 1: the levels were computed with counters in LDS */
  int32_t scheme;            /* SWEEP_SCHEME_* the DAG was built with */
} sweep_dag_info_t;

enum { SWEEP_BOUNDARY_VACUUM = 0, SWEEP_BOUNDARY_PERIODIC = 1 };
enum { SWEEP_FORM_BATCHED = 0, SWEEP_FORM_PLAIN = 1 };
enum { SWEEP_LAW_UPWIND = 0, SWEEP_LAW_EXP = 1 };

typedef struct {
  int32_t boundary;  /* SWEEP_BOUNDARY_*; PERIODIC requires the meshes' face_shift */
  int32_t n_pbc;     /* periodic passes (>= 1); pass 0 starts from zero inflow */
  double albedo;     /* kappa_s / kappa in [0, 1) */
  int32_t n_scat;    /* source iterations (>= 1), starting from J = 0 */
  int32_t form;      /* SWEEP_FORM_BATCHED: every (mesh, direction) in one launch per pass;
                        SWEEP_FORM_PLAIN: one launch per (mesh, direction, group) */
  int32_t block;     /* threads per workgroup of the sweep kernels, 0 = tuned default */
  int32_t ring;      /* LDS ring capacity in tasks (power of two), 0 = tuned default */
  int32_t use_graph; /* 1: run the pass sequence as a captured hipGraph; the first call with
                        a given set of arguments captures and instantiates it (kept with the
                        DAG, at most 8), later calls replay it on `stream` */
  int32_t law;       /* SWEEP_LAW_UPWIND (first-order upwind balance, default) or
                        SWEEP_LAW_EXP (exponential attenuation, see above) */
  int32_t merge;     /* 1: with periodic boundaries and n_scat > 1, run the combined
                        scheme of sec. 2.7: max(n_pbc, n_scat) passes, each taking its
                        scattering source from the previous pass's direction sums and
                        its periodic inflow from the previous pass; 0: n_scat source
                        iterations of n_pbc passes each (every iteration's first pass
                        from zero inflow) */
  int32_t warm_start; /* 1 (periodic only): the first pass takes its periodic inflow
                        from the phi that `saved` holds (the final pass of an earlier
                        call with this DAG and G) instead of zero (sec. 2.7's warm start);
                        requires `saved` */
  double pbc_tol;    /* > 0 (periodic, nested order): the passes of a source iteration
                        stop after the first pass from the second on whose E (below) is
                        below pbc_tol in every cell, group and mesh; n_pbc is then the
                        maximum (sec. 2.7).  Reads E back after every pass, so it
                        synchronises `stream` per pass and cannot be combined with
                        use_graph or merge.  0 = always n_pbc passes */
  int32_t check;     /* 1: synchronise `stream` at the end of the call and return
                        SWEEP_ERR_INVALID_ARG if the kernels met invalid input (see the
                        conventions above); 0: leave it to the next synchronising call */
  int32_t grid;      /* batched form: at most this many persistent workgroups (each takes
                        (mesh, direction) units from a shared counter until none is
                        left); 0 = as many as the GPU holds at once.  Results do not
                        depend on it */
  int32_t pack;      /* batched form: groups swept together by one workgroup (1 to 4);
                        the G groups are cut into chunks of `pack` (and a last chunk of
                        the rest), every (mesh, direction, chunk) a separate work item.
                        0 = the smallest packing dividing G whose work items fit one per
                        compute unit (else 4).  Results do not depend on it */
} sweep_fwd_opts_t;

/* Message of the last failed call on this thread ("" if none). */
const char* sweep_last_error(void);

/* Build the dependency graphs of `n_meshes` meshes for `n_dirs` directions
 * (algorithm 2's upwind counts, sec. 2.5; levels by Kahn's algorithm).
 *   meshes: HOST array of n_meshes descriptors (their arrays on the device)
 *   dirs:   HOST [n_dirs*3] unit vectors (FP64); every direction owns 4pi/n_dirs
 *   opts:   may be NULL for defaults
 * Synchronises `stream` once.  Errors: INVALID_ARG (validation), CYCLE, OOM, HIP,
 * UNSUPPORTED (more than 2^31 - 2 tasks, cells x directions, in one DAG). */
sweep_status_t sweep_build_dag(const sweep_mesh_t* meshes, int32_t n_meshes, const double* dirs,
                               int32_t n_dirs, const sweep_build_opts_t* opts, void* stream,
                               sweep_dag_t* out);

/* Release the DAG and its device buffers (NULL is ignored). */
sweep_status_t sweep_destroy_dag(sweep_dag_t dag);

/* Sizes and critical-path statistics (host struct). */
sweep_status_t sweep_dag_info(sweep_dag_t dag, sweep_dag_info_t* info);

/* Copy the graphs to HOST buffers of n_dirs * n_cells int32 each, laid out
 * [mesh][direction][local cell] (tasks of mesh m start at n_dirs * mesh offset):
 *   level: longest-path level of every task (0 = no upwind dependency);
 *   order: the cells of each (mesh, direction) sorted by (level, cell id);
 *   indeg: number of upwind (graph) dependencies of every task.
 * Any pointer may be NULL.  Synchronises `stream`. */
sweep_status_t sweep_dag_export(sweep_dag_t dag, int32_t* level, int32_t* order, int32_t* indeg,
                                void* stream);

/* Bytes of the `saved` workspace sweep_forward fills for sweep_adjoint:
 * phi of the final pass ([n_dirs][C_total][G] FP32; the exit flux density x
 * under SWEEP_LAW_EXP) followed by the direction sums sum_d phi of every source
 * iteration ([n_scat][C_total][G] FP32) and, with periodic boundaries (nested
 * order), phi of the passes before the last ([n_pbc - 1][n_dirs][C_total][G]
 * FP32) of the last iteration; with warm_start and n_scat > 1, then the inflow
 * the first pass started from ([n_dirs][C_total][G] FP32, for the adjoint's
 * recomputation of that pass); with pbc_tol (nested order, n_pbc > 1), then the
 * number of passes each iteration ran ([n_scat] FP32). */
size_t sweep_saved_bytes(sweep_dag_t dag, int32_t G, const sweep_fwd_opts_t* opts);

/* Forward sweep: n_scat source iterations, each made of n_pbc passes (vacuum:
 * one pass) over every (mesh, direction), groups packed per task.
 *   kappa, emission: DEVICE [C_total][G] FP32, extinction (>= 0) and isotropic
 *                    luminosity (>= 0, photons/s) per cell
 *   J, absorbed:     DEVICE [C_total][G] FP32 outputs of the final pass
 *   totals:          DEVICE [n_meshes][G][8] FP64 outputs of the final pass:
 *                    emitted, absorbed, escaped through vacuum walls, periodic
 *                    inflow, periodic outflow, net scattering source (scattered
 *                    in from the previous iteration minus scattered out), max over
 *                    cells of E = |j_n - j_{n-1}|/(j_n + j_{n-1}) on the per-cell
 *                    periodic inflow j of the last two passes (eq. relativeErrorPbc),
 *                    and the L1 form of E; balance:
 *                    emitted + pbc_in + scat_net = absorbed + escaped + pbc_out
 *   saved:           DEVICE workspace of sweep_saved_bytes() bytes, or NULL
 *   opts:            may be NULL for defaults (vacuum, one pass, no scattering)
 * Errors: INVALID_ARG (with check: also invalid kappa or emission),
 * UNSUPPORTED (a mesh whose cells x G x 4 bytes exceed the kernels' 32-bit
 * buffer range), OOM, HIP. */
sweep_status_t sweep_forward(sweep_dag_t dag, int32_t G, const float* kappa, const float* emission,
                             const sweep_fwd_opts_t* opts, float* J, float* absorbed,
                             double* totals, void* saved, size_t saved_bytes, void* stream);

/* Adjoint sweep (reverse levels over the transposed graphs) for a loss
 * L(J, absorbed): given dL_dJ and dL_dabsorbed (DEVICE [C_total][G] FP32),
 * writes dL_dkappa and dL_demission (DEVICE [C_total][G] FP32).  `saved` must
 * hold what sweep_forward wrote with the same kappa, emission and opts.
 * Source iterations are differentiated with per-iteration recomputation from
 * the saved direction sums.  Periodic passes (nested order) are differentiated
 * pass by pass in reverse: before the reverse sweep of pass p, every task of
 * a periodic cell gets w lambda^{p+1} of the partner cell through each of its
 * periodic outflow faces added to its source (a fixed sequence of FP32 FMAs in
 * face order), so the gradients are the same bits on every run.  The merged
 * order (opts->merge) is differentiated through its single sequence of passes:
 * every pass is recomputed, then reversed with its own source gradient (the
 * loss on the last pass, the scattering source's on the others) and the later
 * pass's lambda through the periodic faces.  A warm start's inflow is held
 * fixed (no gradient flows into it).  With pbc_tol the adjoint runs the passes
 * each iteration ran in the forward call (kept in `saved`; the counts are held
 * fixed); it synchronises `stream` to read them and cannot be captured
 * (use_graph: INVALID_ARG). */
sweep_status_t sweep_adjoint(sweep_dag_t dag, int32_t G, const float* kappa,
                             const float* emission, const sweep_fwd_opts_t* opts,
                             const void* saved, size_t saved_bytes, const float* dL_dJ,
                             const float* dL_dabsorbed, float* dL_dkappa, float* dL_demission,
                             void* stream);

/* Synchronise `stream` and report the invalid input that the kernels of
 * earlier calls on `dag` met (see the conventions above); clears the report.
 * Errors: INVALID_ARG (there was such input), NOT_BUILT, HIP. */
sweep_status_t sweep_sync(sweep_dag_t dag, void* stream);

/* Critical-path length of every (mesh, direction) graph: depth[m * n_dirs + d]
 * (HOST, n_meshes * n_dirs int32), the number of levels, i.e. of steps of a
 * level-synchronous sweep (sec. 2.5's pipe length).  Host data, no sync. */
sweep_status_t sweep_dag_depths(sweep_dag_t dag, int32_t* depth);

/* Tasks per level, summed over the directions of mesh `mesh` (every mesh if
 * mesh = -1): width[l] for l < n_levels (HOST int64; levels past a graph's
 * depth count nothing).  This is how many tasks a level-synchronous sweep has
 * in flight at each step, the GPU analogue of the paper's pipe fill (sec. 2.5).
 * Synchronises `stream`.  Errors: INVALID_ARG, NOT_BUILT, OOM, HIP. */
sweep_status_t sweep_dag_level_widths(sweep_dag_t dag, int32_t mesh, int64_t* width,
                                      int32_t n_levels, void* stream);

/* Autotuner of the sweep's launch shape: times `reps` forward sweeps (after
 * one untimed sweep) of the batched form for every candidate number of threads
 * per workgroup (256, 512, 1024) and LDS ring capacity (a quarter to twice the
 * default, those that fit the LDS), with HIP events on `stream`, and writes
 * into `best` a copy of `opts` (NULL: defaults) with the fastest `block` and
 * `ring`, and into `best_ms` its time per sweep.  The DAG keeps nothing: pass
 * `best` to sweep_forward / sweep_adjoint.  Results of different shapes agree
 * to FP32 rounding (the ring capacity changes the order in which a task's
 * ring misses are added).  Synchronises `stream`.
 * Errors: INVALID_ARG, UNSUPPORTED (nothing fits), HIP. */
sweep_status_t sweep_tune(sweep_dag_t dag, int32_t G, const float* kappa, const float* emission,
                          const sweep_fwd_opts_t* opts, int32_t reps, sweep_fwd_opts_t* best,
                          double* best_ms, void* stream);

/* Hydrogen photoionisation chemistry for time-dependent runs such as the R-type
 * expansion of an HII region (sec. 3.1.1): one frequency bin, constant cross
 * section and case B recombination coefficient (tests section), uniform n_H. */
typedef struct {
  double n_H;         /* hydrogen number density (cm^-3) */
  double sigma_H;     /* photoionisation cross section (cm^2) */
  double alpha_B;     /* case B recombination coefficient (cm^3 s^-1) */
  double photon_rate; /* photons/s per unit of the emission (and absorbed) arrays */
  double length_unit; /* cm per mesh length unit (volumes scale with its cube) */
  double dt_max;      /* largest step (s) */
  double courant;     /* step-limit factor f in (0, 1] */
  double reserved[5];
} sweep_ion_params_t;

/* One chemistry step after a forward sweep with G = 1 (use SWEEP_LAW_EXP and
 * kappa = n_H y sigma_H length_unit, which this call writes for the next sweep):
 *   absorbed: DEVICE [C_total] FP32, the `absorbed` output of sweep_forward
 *             (photons/s in units of photon_rate; albedo 0)
 *   neutral:  DEVICE [C_total] FP64 neutral fraction y in [0, 1], updated in place
 *   kappa:    DEVICE [C_total] FP32 output, n_H y' sigma_H length_unit
 *   t_left:   the step is at most t_left seconds
 *   dt:       HOST output, the step taken (s)
 * With u = 1 - y, V the cell volume in cm^3 and P = photon_rate * absorbed:
 *   dt = min(dt_max, t_left, courant * min_c n_H V y / (P - alpha_B n_H^2 u^2 V))
 * over the cells with a positive denominator, so no cell gains more ionised
 * atoms than it has neutral ones; then every absorbed photon ionises one atom
 * and recombination is implicit:
 *   n_H V (u' - u) = P dt - alpha_B n_H^2 u'^2 V dt   (photon conserving).
 * Synchronises `stream` once (to read the step).  Errors: INVALID_ARG, HIP. */
sweep_status_t sweep_ion_step(sweep_dag_t dag, const float* absorbed, const sweep_ion_params_t* p,
                              double t_left, double* neutral, float* kappa, double* dt,
                              void* stream);

/* sweep_ion_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc): the same
 * arguments, kernels and results, but the per-step minimum it reduces into is a
 * static 8-byte device array of the library (each GPU holds its own copy until
 * the process ends) instead of a buffer allocated with the DAG.  It calls no
 * allocating routine.  One word serves every mesh size, so no input is too
 * large for it.  Every call on a GPU shares that GPU's word: calls that overlap
 * on one GPU (several streams or host threads) race and must be serialised by
 * the caller.  The word is reset by a kernel at the start of each call.
 * Synchronises `stream` once.  Errors: INVALID_ARG, NOT_BUILT, HIP. */
sweep_status_t sweep_ion_step_noalloc(sweep_dag_t dag, const float* absorbed,
                                      const sweep_ion_params_t* p, double t_left, double* neutral,
                                      float* kappa, double* dt, void* stream);

/* The absorption coefficient of the neutral hydrogen for the next sweep of a
 * photoionisation run: kappa[c] = n_H y[c] sigma_H length_unit (DEVICE
 * neutral [C_total] FP64 in, kappa [C_total] FP32 out), the value sweep_ion_step
 * writes after each step; for the first sweep of a run.  Uses n_H, sigma_H and
 * length_unit of `p`.  Errors: INVALID_ARG, NOT_BUILT, HIP. */
sweep_status_t sweep_ion_kappa(sweep_dag_t dag, const sweep_ion_params_t* p, const double* neutral,
                               float* kappa, void* stream);

/* Kernel timing with HIP events (for measurement tools).  While enabled, every
 * launch of the library's main kernels is bracketed by two hipEvents recorded
 * on the launch stream.  Kernel names: "count", "kahn", "fill", "prep",
 * "sweep_fwd", "sweep_adj", "reduce".  sweep_profile_read synchronises on the
 * recorded events and returns the number of launches and their summed
 * duration (ms) since the last reset; unknown names read as zero. */
sweep_status_t sweep_profile_enable(int32_t on);
sweep_status_t sweep_profile_reset(void);
sweep_status_t sweep_profile_read(const char* kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* SWEEP_H_ */

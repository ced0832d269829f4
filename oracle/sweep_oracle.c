/*
 * Plain FP64 CPU oracle of the transport sweep (test infrastructure only).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * use this file.  It shares no code with the GPU library.  Build:
 *   gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 *
 * What it computes (Peter et al. 2022, "The Sweep Method for radiative
 * Transfer in Arepo"):
 *
 *  Orientation (sec. 2.5, appendix A): for direction Omega and the half-face f
 *  of cell c with unit normal n (pointing out of c), s = (Ox nx + Oy ny) + Oz nz
 *  in FP64 without contraction.  s > eps: outflow face (the neighbour is
 *  downwind); s < -eps: inflow face (the neighbour is upwind); otherwise the
 *  face carries no radiation in this direction.  w = A |s|.
 *
 *  Per-cell balance (transport scheme (a) of sec. 2.6 with a first-order
 *  upwind closure): the cell emits through each outflow face i the share
 *  A_i (n_i . Omega) / sum_j A_j (n_j . Omega) of its total outflow, i.e.
 *  w_i phi_c, and
 *      (Aperp_c + kappa_c V_c) phi_c = sum_{inflow faces} w_f phi_upwind + S_c,
 *  Aperp_c = sum of w over outflow faces, S_c = L_c / D (+ scattering source).
 *  Scheme (b) of sec. 2.6 (direction-conserving transport): the same total
 *  outflow Aperp_c phi_c is shared equally by the n outflow faces whose normals
 *  are the most aligned with Omega (n = 3 = the number of dimensions, the
 *  paper's choice), so only those faces carry radiation (see carries()); the
 *  dependency graph keeps only their edges.
 *  Vacuum walls bring no inflow (sec. 2.5, fixed boundaries with I = 0).
 *
 *  Schedule (algorithm 2): Kahn's topological traversal with a FIFO, one per
 *  direction since tasks of different directions never interact (directions
 *  may run on separate threads; results do not depend on it).  A task's level
 *  is 0 without upwind tasks, else 1 + max level of its upwind tasks.
 *
 *  Exponential cell law (the attenuation form 1 - e^{-dn sigma} of the
 *  scattering test, sec. 3.3,
 *  with the mean distance travelled in the cell read as the mean chord
 *  V / Aperp of a parallel beam, so the optical depth is tau = kappa V / Aperp):
 *  the total power entering the task, T = inflow + S, leaves it attenuated by
 *  e^{-tau}, split over the outflow faces in proportion to w, and the rest,
 *  T (1 - e^{-tau}), is absorbed.  The exit flux density (what the downwind
 *  cells and the walls see, per unit w) is T e^{-tau} / Aperp and the cell
 *  average, absorbed / (kappa V), is T (1 - e^{-tau}) / (kappa V) (T / Aperp for
 *  kappa = 0).  tau is capped at TAU_CAP = 40 for the transmission: a thicker
 *  cell passes on e^{-40} = 4.2e-18 of its power, which keeps the exit flux
 *  density of single precision implementations in the normal range; the cap
 *  changes no result by more than that fraction of T and conservation stays
 *  exact.  J and absorbed use the cell average; escape and periodic outflow
 *  use the exit flux density.  Under the first-order upwind law both are phi.
 *
 *  Periodic boundaries (sec. 2.7): faces with a non-zero image shift are cut
 *  from the dependency graph; radiation leaving through them enters the
 *  partner cell in the next pass (pass 0 starts from zero inflow).
 *
 *  Source iteration (sec. 2.3, algorithm 1) with isotropic scattering
 *  (eq. radiativeTransfer): kappa is the extinction, kappa_s = a kappa,
 *  kappa_a = (1-a) kappa; iteration i uses the source
 *  S = L/D + kappa_s V sum_d' avg^{i-1}_{d'} / D, avg^{-1} = 0.
 *
 *  Outputs: J = (1/4pi) sum_d avg, absorbed = kappa_a V sum_d avg (avg: the
 *  cell average, phi itself under the upwind law); totals per
 *  group: [emitted, absorbed, escaped, periodic inflow, periodic outflow,
 *  net scattering source, max E, L1 E] where E is the relative change of the
 *  periodic inflow per cell between the last two passes (eq. relativeErrorPbc).
 *
 *  Adjoint: reverse sweep of the transposed system processed in the reverse
 *  of the recorded queue order; the derivation is in the function comments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_CYCLE -2
#define ORC_ERR_OOM -3
#define ORC_ERR_UNSUPPORTED -6

/* Transport schemes of sec. 2.6 (how a cell's outflow is shared among its
 * downwind faces). */
#define SCHEME_AREA 0    /* (a): in proportion to A_i (n_i . Omega) over every outflow face */
#define SCHEME_ALIGNED 1 /* (b): equally over the n outflow faces whose normals are the most
                            aligned with Omega (direction-conserving transport) */

typedef struct {
  int32_t n_cells;
  const int64_t* face_ptr;
  const int32_t* face_nbr;
  const int8_t* face_shift; /* may be NULL */
  const double* face_area;
  const double* face_normal; /* 3 per face */
  const double* cell_volume;
  const int32_t* face_twin;  /* matching half-face of the neighbour (needed by scheme (b)) */
  int32_t scheme;            /* SCHEME_AREA or SCHEME_ALIGNED */
  int32_t n_aligned;         /* scheme (b): faces that share the outflow (n_dim = 3 in the paper) */
} orc_mesh;

static double orient(const double* om, const double* n) {
  double a = om[0] * n[0];
  double b = om[1] * n[1];
  double c = om[2] * n[2];
  return (a + b) + c;
}

/* face classes */
#define LAW_UPWIND 0
#define LAW_EXP 1
#define TAU_CAP 40.0

/* Exponential law of one task: exit flux density and cell average of the
 * total entering power T (see the header). */
static void exp_law(double T, double aperp, double kV, double* out, double* avg) {
  const double tau = kV / aperp;
  const double tc = tau < TAU_CAP ? tau : TAU_CAP;
  *out = T * exp(-tc) / aperp;
  *avg = kV > 0.0 ? T * (-expm1(-tc)) / kV : T / aperp;
}

#define F_NONE 0
#define F_OUT 1
#define F_IN 2

static int face_class(double s, double eps) {
  if (s > eps) return F_OUT;
  if (s < -eps) return F_IN;
  return F_NONE;
}

static int is_periodic_face(const orc_mesh* m, int64_t f) {
  return m->face_shift != NULL && m->face_shift[f] != 0;
}

/* Does radiation of cell c leave through its face f in direction om, and with
 * which weight w (what leaves is w times the cell's value)?
 *   scheme (a): every outflow face (s > eps), w = A_f |s_f|;
 *   scheme (b): the n outflow faces with the largest s (ties: the lower face
 *     index first), n = min(n_aligned, number of outflow faces), each with
 *     w = Aperp_c / n, Aperp_c = sum over all outflow faces of A |s| (the same
 *     total outflow as scheme (a), shared equally). */
static int carries(const orc_mesh* m, const double* om, double eps, int32_t c, int64_t f,
                   double* w) {
  const double sf = orient(om, m->face_normal + 3 * f);
  if (face_class(sf, eps) != F_OUT) return 0;
  if (m->scheme == SCHEME_AREA) {
    *w = m->face_area[f] * fabs(sf);
    return 1;
  }
  int32_t n_out = 0, rank = 0;
  double aperp = 0.0;
  for (int64_t g = m->face_ptr[c]; g < m->face_ptr[c + 1]; ++g) {
    const double sg = orient(om, m->face_normal + 3 * g);
    if (face_class(sg, eps) != F_OUT) continue;
    ++n_out;
    aperp += m->face_area[g] * fabs(sg);
    if (sg > sf || (sg == sf && g < f)) ++rank;
  }
  const int32_t n = n_out < m->n_aligned ? n_out : m->n_aligned;
  if (rank >= n) return 0;
  *w = aperp / n;
  return 1;
}

/* Does radiation enter cell c through its face f (from the neighbour, interior
 * or periodic), and with which weight?  Scheme (a): f is an inflow face, w the
 * face's own A |s| (equal to its twin's); scheme (b): the neighbour sends
 * through the twin face. */
static int receives(const orc_mesh* m, const double* om, double eps, int32_t c, int64_t f,
                    double* w) {
  const int32_t nb = m->face_nbr[f];
  if (nb < 0) return 0;
  if (m->scheme == SCHEME_AREA) {
    const double s = orient(om, m->face_normal + 3 * f);
    if (face_class(s, eps) != F_IN) return 0;
    *w = m->face_area[f] * fabs(s);
    return 1;
  }
  (void)c;
  return carries(m, om, eps, nb, m->face_twin[f], w);
}

/* in-graph upwind dependency: radiation received through an interior
 * (non-periodic) face */
static int upwind_count(const orc_mesh* m, const double* om, double eps, int32_t c) {
  int n = 0;
  double w;
  for (int64_t f = m->face_ptr[c]; f < m->face_ptr[c + 1]; ++f) {
    if (m->face_nbr[f] < 0 || is_periodic_face(m, f)) continue;
    if (receives(m, om, eps, c, f, &w)) ++n;
  }
  return n;
}

/* Kahn/FIFO traversal of one direction: fills the processing order and levels.
 * Returns the number of processed tasks. */
static int32_t fifo_order(const orc_mesh* m, const double* om, double eps, int32_t* cnt,
                          int32_t* queue, int32_t* level) {
  const int32_t C = m->n_cells;
  int32_t head = 0, tail = 0;
  for (int32_t c = 0; c < C; ++c) {
    cnt[c] = upwind_count(m, om, eps, c);
    level[c] = 0;
    if (cnt[c] == 0) queue[tail++] = c;
  }
  while (head < tail) {
    const int32_t c = queue[head++];
    double w;
    for (int64_t f = m->face_ptr[c]; f < m->face_ptr[c + 1]; ++f) {
      const int32_t nb = m->face_nbr[f];
      if (nb < 0 || is_periodic_face(m, f)) continue;
      if (!carries(m, om, eps, c, f, &w)) continue;
      if (level[nb] < level[c] + 1) level[nb] = level[c] + 1;
      if (--cnt[nb] == 0) queue[tail++] = nb;
    }
  }
  return head;
}

/* ------------------------------------------------------------------ DAG */
/* level, indeg: [D][C]; order: [D][C] cells of each direction sorted by (level, c);
 * depth: [D].  Returns ORC_ERR_CYCLE if some direction cannot be fully ordered. */
int orc_build_dag(const orc_mesh* m, int32_t D, const double* dirs, double eps, int32_t* level,
                  int32_t* order, int32_t* indeg, int32_t* depth) {
  const int32_t C = m->n_cells;
  int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t d = 0; d < D; ++d) {
    const double* om = dirs + 3 * d;
    int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
    int32_t* lv = level + (int64_t)d * C;
    for (int32_t c = 0; c < C; ++c) indeg[(int64_t)d * C + c] = upwind_count(m, om, eps, c);
    int32_t done = fifo_order(m, om, eps, cnt, q, lv);
    if (done != C) {
#pragma omp critical
      status = ORC_ERR_CYCLE;
    } else {
      /* counting sort by level, stable in c */
      int32_t L = 0;
      for (int32_t c = 0; c < C; ++c)
        if (lv[c] + 1 > L) L = lv[c] + 1;
      int32_t* ptr = (int32_t*)calloc((size_t)L + 1, sizeof(int32_t));
      for (int32_t c = 0; c < C; ++c) ptr[lv[c] + 1]++;
      for (int32_t l = 0; l < L; ++l) ptr[l + 1] += ptr[l];
      int32_t* o = order + (int64_t)d * C;
      for (int32_t c = 0; c < C; ++c) o[ptr[lv[c]]++] = c;
      free(ptr);
      depth[d] = L;
    }
    free(cnt);
    free(q);
  }
  return status;
}

/* ------------------------------------------------------------------ forward */
/* One sweep of one direction over all groups.
 *   src:  [C][G] source per task of this direction (already divided by D)
 *   prev: [C][G] phi of this direction in the previous periodic pass (NULL: zero)
 *   phi:  [C][G] output: exit flux density (what downwind cells and walls see)
 *   avg:  [C][G] output: cell average (equal to phi under the upwind law)
 *   acc:  [G][4] += escaped, periodic inflow, periodic outflow (FP64)
 *   jin:  [C][G] += periodic inflow into each cell (may be NULL)
 *   qorder: [C] processing order (output, may be NULL) */
static int sweep_direction(const orc_mesh* m, const double* om, double eps, int32_t G,
                           int32_t law, const double* kappa, const double* src,
                           const double* prev, double* phi, double* avg, double* acc,
                           double* jin, int32_t* cnt, int32_t* queue, int32_t* lvl,
                           int32_t* qorder) {
  const int32_t C = m->n_cells;
  double* nin = (double*)malloc(sizeof(double) * (size_t)G);
  int32_t head = 0, tail = 0;
  for (int32_t c = 0; c < C; ++c) {
    cnt[c] = upwind_count(m, om, eps, c);
    if (cnt[c] == 0) queue[tail++] = c;
  }
  (void)lvl;
  while (head < tail) {
    const int32_t c = queue[head++];
    if (qorder) qorder[head - 1] = c;
    /* solve the task: gather inflow in face order */
    double aperp = 0.0;
    for (int32_t g = 0; g < G; ++g) nin[g] = 0.0;
    for (int64_t f = m->face_ptr[c]; f < m->face_ptr[c + 1]; ++f) {
      const double s = orient(om, m->face_normal + 3 * f);
      double w;
      if (face_class(s, eps) == F_OUT) {
        aperp += m->face_area[f] * fabs(s);
      } else if (receives(m, om, eps, c, f, &w)) {
        const int32_t nb = m->face_nbr[f];
        if (is_periodic_face(m, f)) {
          if (prev)
            for (int32_t g = 0; g < G; ++g) {
              const double in = w * prev[(int64_t)nb * G + g];
              nin[g] += in;
              acc[4 * g + 1] += in;
              if (jin) jin[(int64_t)c * G + g] += in;
            }
        } else {
          for (int32_t g = 0; g < G; ++g) nin[g] += w * phi[(int64_t)nb * G + g];
        }
      }
    }
    for (int32_t g = 0; g < G; ++g) {
      const int64_t i = (int64_t)c * G + g;
      const double kV = kappa[i] * m->cell_volume[c];
      if (law == LAW_EXP) {
        if (!(aperp > 0.0)) {
          free(nin);
          return ORC_ERR_ARG;
        }
        exp_law(nin[g] + src[i], aperp, kV, &phi[i], &avg[i]);
        continue;
      }
      const double den = aperp + kV;
      if (!(den > 0.0)) {
        free(nin);
        return ORC_ERR_ARG;
      }
      phi[i] = (nin[g] + src[i]) / den;
      avg[i] = phi[i];
    }
    /* outflow: boundaries and downwind neighbours */
    for (int64_t f = m->face_ptr[c]; f < m->face_ptr[c + 1]; ++f) {
      double w;
      if (!carries(m, om, eps, c, f, &w)) continue;
      const int32_t nb = m->face_nbr[f];
      if (nb < 0) {
        for (int32_t g = 0; g < G; ++g) acc[4 * g + 0] += w * phi[(int64_t)c * G + g];
      } else if (is_periodic_face(m, f)) {
        for (int32_t g = 0; g < G; ++g) acc[4 * g + 2] += w * phi[(int64_t)c * G + g];
      } else if (--cnt[nb] == 0) {
        queue[tail++] = nb;
      }
    }
  }
  free(nin);
  return head == C ? ORC_OK : ORC_ERR_CYCLE;
}

/* Forward sweep with periodic passes and source iteration.
 *   kappa, emission, J, absorbed: [C][G]
 *   totals: [G][8]
 *   law: LAW_UPWIND or LAW_EXP
 *   merged: 1 = periodic passes and source iterations advance together (see below)
 *   phi_init: [D][C][G] exit flux densities whose periodic outflow feeds the first
 *             pass (a warm start from an earlier solution), or NULL (zero inflow)
 *   pbc_tol: > 0 (nested order only): the periodic passes of an iteration stop after
 *            the first pass (from the second on) whose E is below pbc_tol in every
 *            cell and group; n_pbc is then the maximum (sec. 2.7)
 *   phi_out: [D][C][G] exit flux density of the final pass (may be NULL)
 *   jsum_ckpt: [n_scat][C][G] sum_d of the cell averages of every iteration's
 *              final pass (may be NULL)
 *   qorder: [D][C] FIFO processing order of every direction (may be NULL) */
int orc_forward(const orc_mesh* m, int32_t D, const double* dirs, double eps, int32_t G,
                const double* kappa, const double* emission, int32_t periodic, int32_t n_pbc,
                double albedo, int32_t n_scat, int32_t law, int32_t merged,
                const double* phi_init, double pbc_tol, double* J, double* absorbed,
                double* totals, double* phi_out, double* jsum_ckpt, int32_t* qorder) {
  const int32_t C = m->n_cells;
  const int64_t CG = (int64_t)C * G;
  if (D < 1 || G < 1 || n_pbc < 1 || n_scat < 1 || albedo < 0.0 || albedo >= 1.0) return ORC_ERR_ARG;
  if (law != LAW_UPWIND && law != LAW_EXP) return ORC_ERR_ARG;
  if (!(pbc_tol >= 0.0) || (merged && pbc_tol > 0.0)) return ORC_ERR_ARG;
  if (!periodic) n_pbc = 1;
  double* phi = (double*)calloc((size_t)(D * CG), sizeof(double));
  double* avg = (double*)calloc((size_t)(D * CG), sizeof(double));
  double* phiprev = (double*)calloc((size_t)(D * CG), sizeof(double));
  double* jsum = (double*)calloc((size_t)CG, sizeof(double));     /* sum_d phi, current */
  double* jsum_old = (double*)calloc((size_t)CG, sizeof(double)); /* previous iteration */
  double* src = (double*)calloc((size_t)CG, sizeof(double));
  double* jin = (double*)calloc((size_t)(D * CG), sizeof(double));
  double* jin_old = (double*)calloc((size_t)CG, sizeof(double));
  double* accd = (double*)calloc((size_t)D * 4 * G, sizeof(double));
  if (!phi || !avg || !phiprev || !jsum || !jsum_old || !src || !jin || !jin_old || !accd)
    return ORC_ERR_OOM;
  int status = ORC_OK;
  /* merged: one sequence of max(n_pbc, n_scat) passes, each taking its scattering
   * source from the previous pass's direction sums and its periodic inflow from
   * the previous pass (only differs from the nested order with periodic
   * boundaries and several source iterations) */
  const int32_t merge = merged && periodic && n_scat > 1;
  const int32_t n_outer = merge ? 1 : n_scat;
  const int32_t n_inner = merge ? (n_pbc > n_scat ? n_pbc : n_scat) : n_pbc;
  const int32_t warm = periodic && phi_init != NULL;
  int32_t n_done = n_inner; /* passes of the last iteration (fewer if pbc_tol stopped them) */
  for (int32_t it = 0; it < n_outer && status == ORC_OK; ++it) {
    n_done = n_inner;
    if (warm && it == 0)
      memcpy(phiprev, phi_init, sizeof(double) * (size_t)(D * CG));
    else
      memset(phiprev, 0, sizeof(double) * (size_t)(D * CG));
    for (int32_t p = 0; p < n_inner && status == ORC_OK; ++p) {
      /* source of this iteration (nested: once per iteration; merged: every pass) */
      if (p == 0 || merge)
        for (int32_t c = 0; c < C; ++c)
          for (int32_t g = 0; g < G; ++g) {
            const int64_t i = (int64_t)c * G + g;
            const double ks = albedo * kappa[i];
            src[i] = emission[i] / D + ks * m->cell_volume[c] * jsum_old[i] / D;
          }
      /* keep the previous pass's per-cell periodic inflow for E */
      if (p > 0) {
        for (int64_t i = 0; i < CG; ++i) {
          double s = 0.0;
          for (int32_t d = 0; d < D; ++d) s += jin[(int64_t)d * CG + i];
          jin_old[i] = s;
        }
      }
      memset(jin, 0, sizeof(double) * (size_t)(D * CG));
      memset(accd, 0, sizeof(double) * (size_t)D * 4 * G);
#pragma omp parallel for schedule(dynamic, 1)
      for (int32_t d = 0; d < D; ++d) {
        int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
        int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
        int st = sweep_direction(m, dirs + 3 * d, eps, G, law, kappa, src,
                                 (periodic && (p > 0 || (warm && it == 0)))
                                     ? phiprev + (int64_t)d * CG
                                     : NULL,
                                 phi + (int64_t)d * CG, avg + (int64_t)d * CG,
                                 accd + (int64_t)d * 4 * G,
                                 jin + (int64_t)d * CG, cnt, q, NULL,
                                 qorder ? qorder + (int64_t)d * C : NULL);
        if (st != ORC_OK) {
#pragma omp critical
          status = st;
        }
        free(cnt);
        free(q);
      }
      if (status != ORC_OK) break;
      /* convergence test of sec. 2.7: stop once E < pbc_tol in every cell and group */
      int stop = 0;
      if (periodic && pbc_tol > 0.0 && p > 0) {
        double emax = 0.0;
        for (int64_t i = 0; i < CG; ++i) {
          double jn = 0.0;
          for (int32_t d = 0; d < D; ++d) jn += jin[(int64_t)d * CG + i];
          const double jo = jin_old[i];
          const double e = jn + jo > 0.0 ? fabs(jn - jo) / (jn + jo) : 0.0;
          if (e > emax) emax = e;
        }
        stop = emax < pbc_tol;
      }
      if (p + 1 < n_inner && !stop) memcpy(phiprev, phi, sizeof(double) * (size_t)(D * CG));
      if (merge || p + 1 == n_inner || stop) {
        /* direction sum of the cell averages in ascending d */
        for (int64_t i = 0; i < CG; ++i) {
          double s = 0.0;
          for (int32_t d = 0; d < D; ++d) s += avg[(int64_t)d * CG + i];
          jsum[i] = s;
        }
      }
      if (merge && p + 1 < n_inner) memcpy(jsum_old, jsum, sizeof(double) * (size_t)CG);
      if (stop) {
        n_done = p + 1;
        break;
      }
    }
    if (status != ORC_OK) break;
    /* merged: the sums of the final pass go to the last checkpoint */
    const int32_t slot = merge ? n_scat - 1 : it;
    if (jsum_ckpt) memcpy(jsum_ckpt + (int64_t)slot * CG, jsum, sizeof(double) * (size_t)CG);
    if (!merge && it + 1 < n_scat) memcpy(jsum_old, jsum, sizeof(double) * (size_t)CG);
  }
  if (status == ORC_OK) {
    for (int32_t g = 0; g < G; ++g)
      for (int k = 0; k < 8; ++k) totals[8 * g + k] = 0.0;
    for (int32_t c = 0; c < C; ++c)
      for (int32_t g = 0; g < G; ++g) {
        const int64_t i = (int64_t)c * G + g;
        const double V = m->cell_volume[c];
        const double ka = (1.0 - albedo) * kappa[i];
        const double ks = albedo * kappa[i];
        J[i] = jsum[i] / (4.0 * M_PI);
        absorbed[i] = ka * V * jsum[i];
        totals[8 * g + 0] += emission[i];
        totals[8 * g + 1] += absorbed[i];
        /* net scattering source of the last iteration: scattered in - scattered out */
        totals[8 * g + 5] += ks * V * (n_scat > 1 ? jsum_old[i] : 0.0) - ks * V * jsum[i];
        /* periodic-inflow change between the last two passes */
        double jn = 0.0;
        for (int32_t d = 0; d < D; ++d) jn += jin[(int64_t)d * CG + i];
        const double jo = jin_old[i];
        if (periodic && n_done > 1 && jn + jo > 0.0) {
          const double e = fabs(jn - jo) / (jn + jo);
          if (e > totals[8 * g + 6]) totals[8 * g + 6] = e;
        }
        totals[8 * g + 7] += fabs(jn - jo);
        jin_old[i] = jn + jo; /* reuse as denominator accumulator */
      }
    for (int32_t g = 0; g < G; ++g) {
      double den = 0.0;
      for (int32_t c = 0; c < C; ++c) den += jin_old[(int64_t)c * G + g];
      totals[8 * g + 7] = (periodic && n_done > 1 && den > 0.0) ? totals[8 * g + 7] / den : 0.0;
      for (int32_t d = 0; d < D; ++d) {
        totals[8 * g + 2] += accd[(int64_t)d * 4 * G + 4 * g + 0];
        totals[8 * g + 3] += accd[(int64_t)d * 4 * G + 4 * g + 1];
        totals[8 * g + 4] += accd[(int64_t)d * 4 * G + 4 * g + 2];
      }
    }
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * (size_t)(D * CG));
  }
  free(phi);
  free(avg);
  free(phiprev);
  free(jsum);
  free(jsum_old);
  free(src);
  free(jin);
  free(jin_old);
  free(accd);
  return status;
}

/* ------------------------------------------------------------------ adjoint */
/* Derivative of h(tau) = (e^tau - 1) / tau: a Taylor series below 1e-2
 * (truncation below 1.3e-13 relative), the closed form above. */
static double dh_dtau(double tau) {
  if (tau < 1e-2) return 0.5 + tau * (1.0 / 3.0 + tau * (1.0 / 8.0 + tau * (1.0 / 30.0 + tau / 144.0)));
  return ((tau - 1.0) * exp(tau) + 1.0) / (tau * tau);
}

/* Reverse sweep of one direction.  Written with x the stored per-task value
 * (phi under the upwind law, the exit flux density under the exponential law),
 * the forward sweep solves M x = S with M = diag(den) - W (W[c][u] = w of the
 * inflow face of c from u):
 *   upwind:      den = Aperp + kappa V, and the cell average is x;
 *   exponential: den = Aperp e^{tau_c} (T = den x), and the cell average is
 *                r x with r = Aperp (e^{tau_c} - 1) / (kappa V) (1 at kappa = 0),
 *                tau_c = min(tau, TAU_CAP).
 * For g = dL/d(cell average), dL/dx = r g, so lambda = M^{-T} (r g):
 *   lambda_c = (r_c g_c + sum_{outflow faces to interior e} w lambda_e) / den_c,
 * visiting the cells in the reverse of the forward queue order, so every
 * downwind lambda is final before it is read.  With periodic passes the
 * forward pass p also takes w x^{p-1}(partner) through every periodic inflow
 * face, so lambda^p gets w lambda^{p+1}(partner) through every periodic outflow
 * face (lam_next; NULL for the last pass), and only the last pass carries the
 * loss (g = NULL before it).  It also writes, per task,
 *   dk_c = -lambda_c x_c d(den_c)/dkappa_c + g_c x_c dr_c/dkappa_c
 * (the part of dL/dkappa_c this direction contributes through M and r):
 *   upwind: d(den)/dkappa = V, dr/dkappa = 0;
 *   exponential, tau < TAU_CAP: d(den)/dkappa = V e^tau, r = h(tau) with
 *     h(t) = (e^t - 1)/t, dr/dkappa = h'(tau) V / Aperp;
 *   exponential, tau >= TAU_CAP: d(den)/dkappa = 0, dr/dkappa = -r / kappa. */
static void adjoint_direction(const orc_mesh* m, const double* om, double eps, int32_t G,
                              int32_t law, const double* kappa, const double* g,
                              const double* lam_next, const double* x, const int32_t* qorder,
                              double* lam, double* dk) {
  const int32_t C = m->n_cells;
  for (int32_t k = C - 1; k >= 0; --k) {
    const int32_t c = qorder[k];
    const double V = m->cell_volume[c];
    double aperp = 0.0;
    for (int64_t f = m->face_ptr[c]; f < m->face_ptr[c + 1]; ++f) {
      const double s = orient(om, m->face_normal + 3 * f);
      if (face_class(s, eps) == F_OUT) aperp += m->face_area[f] * fabs(s);
    }
    for (int32_t gg = 0; gg < G; ++gg) {
      const int64_t i = (int64_t)c * G + gg;
      const double kap = kappa[i];
      double den, r = 1.0, dden = V, dr = 0.0;
      if (law == LAW_EXP) {
        const double tau = kap * V / aperp;
        if (tau < TAU_CAP) {
          den = aperp * exp(tau);
          r = kap > 0.0 ? aperp * expm1(tau) / (kap * V) : 1.0;
          dden = V * exp(tau);
          dr = dh_dtau(tau) * V / aperp;
        } else {
          den = aperp * exp(TAU_CAP);
          r = aperp * expm1(TAU_CAP) / (kap * V);
          dden = 0.0;
          dr = -r / kap;
        }
      } else {
        den = aperp + kap * V;
      }
      double acc = g ? r * g[i] : 0.0;
      for (int64_t f = m->face_ptr[c]; f < m->face_ptr[c + 1]; ++f) {
        const int32_t nb = m->face_nbr[f];
        double w;
        if (nb < 0 || !carries(m, om, eps, c, f, &w)) continue;
        if (!is_periodic_face(m, f))
          acc += w * lam[(int64_t)nb * G + gg];
        else if (lam_next)  /* what leaves here enters nb in the next pass */
          acc += w * lam_next[(int64_t)nb * G + gg];
      }
      lam[i] = acc / den;
      dk[i] = -lam[i] * x[i] * dden + (g ? g[i] * x[i] * dr : 0.0);
    }
  }
}

/* The merged order (periodic boundaries with n_scat > 1 and `merged`): one
 * sequence of P = max(n_pbc, n_scat) passes, pass p taking its scattering
 * source from the direction sums of pass p-1 and its periodic inflow from pass
 * p-1 (pass 0 from zero inflow and no scattering), the loss on the last pass:
 *   x^p = M^{-1}(S^p + B x^{p-1}),  S^p = L/D + a kappa V jsum^{p-1} / D.
 * Reverse, p = P-1..0:
 *   lambda^p_d = M_d^{-T}(r_d g^p + B^T lambda^{p+1}),
 *   g^{P-1} = the loss's cell-average gradient, g^{p-1} = a kappa V sum_d lambda^p_d / D;
 *   dL/dL += sum_d lambda^p_d / D;
 *   dL/dkappa += sum_d dk^p_d + a V (sum_d lambda^p_d) jsum^{p-1} / D  (jsum^{-1} = 0),
 * plus the loss's own gA (1-a) V jsum^{P-1}.  Every pass is recomputed forward
 * first, keeping its exit values and direction sums. */
static int adjoint_merged(const orc_mesh* m, int32_t D, const double* dirs, double eps, int32_t G,
                          const double* kappa, const double* emission, int32_t P, double albedo,
                          int32_t law, const double* phi_init, const double* gJ, const double* gA,
                          double* dkappa, double* demission) {
  const int32_t C = m->n_cells;
  const int64_t CG = (int64_t)C * G;
  const int64_t DCG = (int64_t)D * CG;
  double* xs = (double*)malloc(sizeof(double) * (size_t)(P * DCG));  /* x of every pass */
  double* js = (double*)malloc(sizeof(double) * (size_t)(P * CG));   /* its direction sums */
  double* avg = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* lam = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* lam_next = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* dkd = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* gsrc = (double*)malloc(sizeof(double) * (size_t)CG);
  double* src = (double*)malloc(sizeof(double) * (size_t)CG);
  int32_t* qorder = (int32_t*)malloc(sizeof(int32_t) * (size_t)D * C);
  int status = ORC_OK;
  if (!xs || !js || !avg || !lam || !lam_next || !dkd || !gsrc || !src || !qorder) status = ORC_ERR_OOM;
  for (int32_t p = 0; p < P && status == ORC_OK; ++p) {
    for (int32_t c = 0; c < C; ++c)
      for (int32_t g = 0; g < G; ++g) {
        const int64_t i = (int64_t)c * G + g;
        const double prev = p > 0 ? js[(int64_t)(p - 1) * CG + i] : 0.0;
        src[i] = emission[i] / D + albedo * kappa[i] * m->cell_volume[c] * prev / D;
      }
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t d = 0; d < D; ++d) {
      int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
      int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
      double acc[4 * 64];
      double* a4 = G <= 64 ? acc : (double*)malloc(sizeof(double) * 4 * (size_t)G);
      memset(a4, 0, sizeof(double) * 4 * (size_t)G);
      const double* prev = p > 0 ? xs + (int64_t)(p - 1) * DCG + (int64_t)d * CG
                           : phi_init ? phi_init + (int64_t)d * CG : NULL;
      int st = sweep_direction(m, dirs + 3 * d, eps, G, law, kappa, src, prev,
                               xs + (int64_t)p * DCG + (int64_t)d * CG, avg + (int64_t)d * CG, a4,
                               NULL, cnt, q, NULL, qorder + (int64_t)d * C);
      if (st != ORC_OK) {
#pragma omp critical
        status = st;
      }
      if (a4 != acc) free(a4);
      free(cnt);
      free(q);
    }
    for (int64_t i = 0; i < CG; ++i) {
      double sum = 0.0;
      for (int32_t d = 0; d < D; ++d) sum += avg[(int64_t)d * CG + i];
      js[(int64_t)p * CG + i] = sum;
    }
  }
  if (status == ORC_OK) {
    memset(dkappa, 0, sizeof(double) * (size_t)CG);
    memset(demission, 0, sizeof(double) * (size_t)CG);
    for (int32_t c = 0; c < C; ++c)
      for (int32_t g = 0; g < G; ++g) {
        const int64_t i = (int64_t)c * G + g;
        const double V = m->cell_volume[c];
        gsrc[i] = gJ[i] / (4.0 * M_PI) + gA[i] * (1.0 - albedo) * kappa[i] * V;
        dkappa[i] += gA[i] * (1.0 - albedo) * V * js[(int64_t)(P - 1) * CG + i];
      }
    for (int32_t p = P - 1; p >= 0; --p) {
#pragma omp parallel for schedule(dynamic, 1)
      for (int32_t d = 0; d < D; ++d)
        adjoint_direction(m, dirs + 3 * d, eps, G, law, kappa, gsrc,
                          p < P - 1 ? lam_next + (int64_t)d * CG : NULL,
                          xs + (int64_t)p * DCG + (int64_t)d * CG, qorder + (int64_t)d * C,
                          lam + (int64_t)d * CG, dkd + (int64_t)d * CG);
      for (int32_t c = 0; c < C; ++c)
        for (int32_t g = 0; g < G; ++g) {
          const int64_t i = (int64_t)c * G + g;
          const double V = m->cell_volume[c];
          double ls = 0.0, dks = 0.0;
          for (int32_t d = 0; d < D; ++d) {
            ls += lam[(int64_t)d * CG + i];
            dks += dkd[(int64_t)d * CG + i];
          }
          const double prev = p > 0 ? js[(int64_t)(p - 1) * CG + i] : 0.0;
          demission[i] += ls / D;
          dkappa[i] += dks + albedo * V * ls * prev / D;
          gsrc[i] = albedo * kappa[i] * V * ls / D;  /* the source gradient of pass p - 1 */
        }
      double* t = lam_next;
      lam_next = lam;
      lam = t;
    }
  }
  free(xs);
  free(js);
  free(avg);
  free(lam);
  free(lam_next);
  free(dkd);
  free(gsrc);
  free(src);
  free(qorder);
  return status;
}

/* Gradients of a loss L(J, absorbed) given gJ = dL/dJ and gA = dL/dabsorbed ([C][G]).
 * avg denotes the cell average and x the stored value of adjoint_direction.
 *
 * Without scattering (one iteration): dL/d avg_{c,d} = gJ_c/(4pi) + gA_c kappa_a,c V_c =: g_c,
 *   lambda_d = M_d^{-T} (r_d g), dL/dL_c = sum_d lambda_{c,d}/D,
 *   dL/dkappa_c = gA_c (1-a) V_c sum_d avg_{c,d} + sum_d dk_{c,d}
 *   (dk from adjoint_direction; under the upwind law sum_d dk = -V_c sum_d lambda phi).
 * With source iteration (iterations i = 0..n-1, outputs from the last):
 *   lambda^{n-1} from g as above; lambda^{i-1}_d = M_d^{-T} (r_d g^{i-1}) with
 *   g^{i-1}_c = a kappa_c V_c (sum_d lambda^i_{c,d}) / D;
 *   dL/dL_c = sum_i sum_d lambda^i_{c,d} / D;
 *   dL/dkappa_c = gA_c (1-a) V_c sum_d avg^{n-1}_{c,d}
 *     + sum_i [ sum_d dk^i_{c,d} + a V_c (sum_d lambda^i_{c,d}) (sum_d' avg^{i-1}_{c,d'}) / D ],
 *   avg^{-1} = 0.
 * With periodic boundaries every iteration is n_pbc passes x^0..x^{P-1} (pass 0
 * from zero inflow, the scattering source the same in every pass, the loss and
 * the next iteration's source on the last pass only).  The reverse passes run
 * p = P-1..0 with lambda^{P-1} from the iteration's adjoint source and lambda^p
 * fed by lambda^{p+1} through the periodic faces (adjoint_direction); the sums
 * over d above become sums over passes and d, each pass's dk using its own x^p.
 * x^p is recomputed from the stored direction sums of iteration i-1. */
int orc_adjoint(const orc_mesh* m, int32_t D, const double* dirs, double eps, int32_t G,
                const double* kappa, const double* emission, int32_t periodic, int32_t n_pbc,
                double albedo, int32_t n_scat, int32_t law, int32_t merged, const double* phi_init,
                double pbc_tol, const double* gJ, const double* gA, double* dkappa,
                double* demission) {
  if (D < 1 || G < 1 || n_scat < 1 || n_pbc < 1 || albedo < 0.0 || albedo >= 1.0) return ORC_ERR_ARG;
  if (!(pbc_tol >= 0.0) || (merged && pbc_tol > 0.0)) return ORC_ERR_ARG;
  if (law != LAW_UPWIND && law != LAW_EXP) return ORC_ERR_ARG;
  if (merged && periodic && n_scat > 1)
    return adjoint_merged(m, D, dirs, eps, G, kappa, emission, n_pbc > n_scat ? n_pbc : n_scat,
                          albedo, law, periodic ? phi_init : NULL, gJ, gA, dkappa, demission);
  if (!periodic) phi_init = NULL;
  const int32_t P = periodic ? n_pbc : 1;
  const int32_t C = m->n_cells;
  const int64_t CG = (int64_t)C * G;
  const int64_t DCG = (int64_t)D * CG;
  double* J = (double*)malloc(sizeof(double) * (size_t)CG);
  double* Ab = (double*)malloc(sizeof(double) * (size_t)CG);
  double tot[8 * 64];
  double* tots = G <= 64 ? tot : (double*)malloc(sizeof(double) * 8 * (size_t)G);
  double* jsum = (double*)malloc(sizeof(double) * (size_t)(n_scat * CG));
  double* xs = (double*)malloc(sizeof(double) * (size_t)(P * DCG)); /* x of every pass */
  double* avg = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* lam = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* lam_next = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* dkd = (double*)malloc(sizeof(double) * (size_t)DCG);
  double* gsrc = (double*)malloc(sizeof(double) * (size_t)CG);
  double* src = (double*)malloc(sizeof(double) * (size_t)CG);
  double* lsum = (double*)malloc(sizeof(double) * (size_t)CG);
  double* dksum = (double*)malloc(sizeof(double) * (size_t)CG);
  int32_t* qorder = (int32_t*)malloc(sizeof(int32_t) * (size_t)D * C);
  /* with pbc_tol: each pass's periodic inflow per direction and, summed over
   * directions, the previous pass's (the stopping test of the forward) */
  const int32_t tol = periodic && pbc_tol > 0.0;
  double* jin = tol ? (double*)malloc(sizeof(double) * (size_t)DCG) : NULL;
  double* jin_old = tol ? (double*)malloc(sizeof(double) * (size_t)CG) : NULL;
  if (!J || !Ab || !tots || !jsum || !xs || !avg || !lam || !lam_next || !dkd || !gsrc || !src ||
      !lsum || !dksum || !qorder || (tol && (!jin || !jin_old)))
    return ORC_ERR_OOM;
  int status = orc_forward(m, D, dirs, eps, G, kappa, emission, periodic, P, albedo, n_scat, law,
                           0, phi_init, pbc_tol, J, Ab, tots, NULL, jsum, NULL);
  if (status == ORC_OK) {
    memset(dkappa, 0, sizeof(double) * (size_t)CG);
    memset(demission, 0, sizeof(double) * (size_t)CG);
    for (int32_t c = 0; c < C; ++c)
      for (int32_t g = 0; g < G; ++g) {
        const int64_t i = (int64_t)c * G + g;
        const double V = m->cell_volume[c];
        gsrc[i] = gJ[i] / (4.0 * M_PI) + gA[i] * (1.0 - albedo) * kappa[i] * V;
        dkappa[i] += gA[i] * (1.0 - albedo) * V * jsum[(int64_t)(n_scat - 1) * CG + i];
      }
    for (int32_t it = n_scat - 1; it >= 0 && status == ORC_OK; --it) {
      /* recompute the passes x^0..x^{P-1} of iteration it from the sums of it-1 */
      for (int32_t c = 0; c < C; ++c)
        for (int32_t g = 0; g < G; ++g) {
          const int64_t i = (int64_t)c * G + g;
          const double prev = it > 0 ? jsum[(int64_t)(it - 1) * CG + i] : 0.0;
          src[i] = emission[i] / D + albedo * kappa[i] * m->cell_volume[c] * prev / D;
        }
      /* passes of this iteration: P, or fewer where pbc_tol stopped the forward
       * (the same test on the same values) */
      int32_t Pit = P;
      if (tol) memset(jin, 0, sizeof(double) * (size_t)DCG);
      for (int32_t p = 0; p < P && status == ORC_OK; ++p) {
        if (tol && p > 0) {
          for (int64_t i = 0; i < CG; ++i) {
            double sum = 0.0;
            for (int32_t d = 0; d < D; ++d) sum += jin[(int64_t)d * CG + i];
            jin_old[i] = sum;
          }
          memset(jin, 0, sizeof(double) * (size_t)DCG);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t d = 0; d < D; ++d) {
          int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
          int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
          double acc[4 * 64];
          double* a4 = G <= 64 ? acc : (double*)malloc(sizeof(double) * 4 * (size_t)G);
          memset(a4, 0, sizeof(double) * 4 * (size_t)G);
          /* warm start: the first pass of the first iteration takes its periodic
           * inflow from phi_init (held fixed: no gradient flows into it) */
          const double* prev = p > 0 ? xs + (int64_t)(p - 1) * DCG + (int64_t)d * CG
                               : (phi_init && it == 0) ? phi_init + (int64_t)d * CG : NULL;
          int st = sweep_direction(m, dirs + 3 * d, eps, G, law, kappa, src, prev,
                                   xs + (int64_t)p * DCG + (int64_t)d * CG, avg + (int64_t)d * CG,
                                   a4, tol ? jin + (int64_t)d * CG : NULL, cnt, q, NULL,
                                   qorder + (int64_t)d * C);
          if (st != ORC_OK) {
#pragma omp critical
            status = st;
          }
          if (a4 != acc) free(a4);
          free(cnt);
          free(q);
        }
        if (status == ORC_OK && tol && p > 0) {
          double emax = 0.0;
          for (int64_t i = 0; i < CG; ++i) {
            double jn = 0.0;
            for (int32_t d = 0; d < D; ++d) jn += jin[(int64_t)d * CG + i];
            const double jo = jin_old[i];
            const double e = jn + jo > 0.0 ? fabs(jn - jo) / (jn + jo) : 0.0;
            if (e > emax) emax = e;
          }
          if (emax < pbc_tol) {
            Pit = p + 1;
            break;
          }
        }
      }
      if (status != ORC_OK) break;
      /* reverse passes */
      memset(lsum, 0, sizeof(double) * (size_t)CG);
      memset(dksum, 0, sizeof(double) * (size_t)CG);
      for (int32_t p = Pit - 1; p >= 0; --p) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t d = 0; d < D; ++d)
          adjoint_direction(m, dirs + 3 * d, eps, G, law, kappa, p == Pit - 1 ? gsrc : NULL,
                            p < Pit - 1 ? lam_next + (int64_t)d * CG : NULL,
                            xs + (int64_t)p * DCG + (int64_t)d * CG, qorder + (int64_t)d * C,
                            lam + (int64_t)d * CG, dkd + (int64_t)d * CG);
        for (int64_t i = 0; i < CG; ++i) {
          double ls = 0.0, dks = 0.0;
          for (int32_t d = 0; d < D; ++d) {
            ls += lam[(int64_t)d * CG + i];
            dks += dkd[(int64_t)d * CG + i];
          }
          lsum[i] += ls;
          dksum[i] += dks;
        }
        double* t = lam_next;
        lam_next = lam;
        lam = t;
      }
      for (int32_t c = 0; c < C; ++c)
        for (int32_t g = 0; g < G; ++g) {
          const int64_t i = (int64_t)c * G + g;
          const double V = m->cell_volume[c];
          const double prev = it > 0 ? jsum[(int64_t)(it - 1) * CG + i] : 0.0;
          demission[i] += lsum[i] / D;
          dkappa[i] += dksum[i] + albedo * V * lsum[i] * prev / D;
        }
      /* adjoint source of the previous iteration */
      for (int32_t c = 0; c < C; ++c)
        for (int32_t g = 0; g < G; ++g) {
          const int64_t i = (int64_t)c * G + g;
          gsrc[i] = albedo * kappa[i] * m->cell_volume[c] * lsum[i] / D;
        }
    }
  }
  free(J);
  free(Ab);
  if (tots != tot) free(tots);
  free(jsum);
  free(xs);
  free(avg);
  free(lam);
  free(lam_next);
  free(dkd);
  free(gsrc);
  free(src);
  free(lsum);
  free(dksum);
  free(qorder);
  free(jin);
  free(jin_old);
  return status;
}

/* Number of OpenMP threads the parallel loops above use. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the number of OpenMP threads of the loops above (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

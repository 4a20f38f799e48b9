/*
 * Kino-PAX CPU oracle -- TEST INFRASTRUCTURE ONLY (see kpo.h).
 *
 * Written from the paper, sequentially and in the paper's order:
 *   Alg. 1  main loop: tree rooted at x_init, V_E = {x_init}, P_accept = 1,
 *           then Propagate -> UpdateEstimates -> UpdateNodeSets until a goal
 *           node appears or the budget runs out.
 *   Alg. 2  Propagate: every frontier node is expanded lambda times with a
 *           random control; the end state is mapped to its sub-region; a valid
 *           segment increments n_valid and is accepted if its sub-region is
 *           unvisited or with probability P_accept; an invalid one increments
 *           n_invalid.
 *   Alg. 3  UpdateEstimates over R_avail: FreeVol (eq. 3), Cov, Score
 *           (eq. 4), then P_accept (eq. 5).
 *   Alg. 4  UpdateNodeSets: V_E -> V_O with probability 1 - P_accept, V_U ->
 *           V_E and the tree with the goal test, V_O -> V_E with probability
 *           P_accept.
 *   eq. 6   lambda = min(lambda_max, floor((t_e - |T|) / |V_E|)).
 * Readings of points the paper leaves open are stated where they are used.
 *
 * Build: gcc -O2 -std=gnu99 -ffp-contract=off -fopenmp -fPIC -shared kpo.c -lm
 * (without -fopenmp the lanes run on one thread; the results are the same).
 */
#include "kpo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies and a    */
/* word permutation, with a Weyl-sequence key schedule.                      */
/* ------------------------------------------------------------------------ */
void kpo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Sampled control component: the top 24 bits of a word as a fraction
 * r in [0, 1), then lo + (hi - lo) * r rounded once (FP32 fused multiply-add).
 * Alg. 2 samples u uniformly from U; the generator is not specified. */
float kpo_control_map(uint32_t w, float lo, float hi) {
  float d = hi - lo;
  float r = (float)(w >> 8) * 0x1p-24f;
  return fmaf(d, r, lo);
}

/* Draw words for expansion (it, parent, sample): controls then acceptance.
 * Counter = (iteration, node, sample, tag); key = seed. */
static void draw_expansion(const kpo_problem* pb, int m, uint32_t it, uint32_t f, uint32_t s,
                           float* u, uint32_t* w_acc) {
  uint32_t key[2] = {(uint32_t)pb->seed, (uint32_t)(pb->seed >> 32)};
  uint32_t ctr[4] = {it, f, s, 0u};
  uint32_t w[4];
  kpo_philox4x32_10(ctr, key, w);
  for (int j = 0; j < m; ++j) u[j] = kpo_control_map(w[j], pb->u_lo[j], pb->u_hi[j]);
  if (m < 4) {
    *w_acc = w[3];
  } else {
    uint32_t ctr1[4] = {it, f, s, 1u};
    uint32_t w1[4];
    kpo_philox4x32_10(ctr1, key, w1);
    *w_acc = w1[0];
  }
}

/* Alg. 2 draws the segment duration dt in (0, T_prop].  With dur_mode = 1
 * it is k steps of h, k uniform in {1 .. K} (T_prop = K h), from word 1 of
 * the counter (it, f, s, 1); with dur_mode = 0 every segment is K steps. */
int32_t kpo_segment_steps(const kpo_problem* pb, uint32_t it, uint32_t f, uint32_t s) {
  if (!pb->dur_mode) return pb->steps;
  uint32_t key[2] = {(uint32_t)pb->seed, (uint32_t)(pb->seed >> 32)};
  uint32_t ctr[4] = {it, f, s, 1u};
  uint32_t w[4];
  kpo_philox4x32_10(ctr, key, w);
  return 1 + (int32_t)(((uint64_t)w[1] * (uint64_t)pb->steps) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Dynamics, eq. (1).                                                        */
/* ------------------------------------------------------------------------ */
/* 6D double integrator: state (p, v), control a: p' = v, v' = a.
 * 12D quadcopter (Newton-Euler rigid body, ZYX Euler angles):
 *   state (p, phi theta psi, v (inertial), p q r (body rates)),
 *   control (thrust T, torques tx ty tz),
 *   p'   = v
 *   v'   = (T / m) * (third column of R(phi, theta, psi)) - g e3
 *   Theta' = W(phi, theta) * omega,
 *            W = [[1, s_phi t_th, c_phi t_th], [0, c_phi, -s_phi],
 *                 [0, s_phi / c_th, c_phi / c_th]]
 *   omega' = I^-1 (tau - omega x I omega),  I = diag(Ixx, Iyy, Izz). */
void kpo_deriv(const kpo_problem* pb, const double* x, const double* u, double* dx) {
  if (pb->dyn == KPO_DI6) {
    dx[0] = x[3]; dx[1] = x[4]; dx[2] = x[5];
    dx[3] = u[0]; dx[4] = u[1]; dx[5] = u[2];
    return;
  }
  const double mass = pb->prm[0], g = pb->prm[1];
  const double Ixx = pb->prm[2], Iyy = pb->prm[3], Izz = pb->prm[4];
  const double phi = x[3], th = x[4], psi = x[5];
  const double P = x[9], Q = x[10], Rr = x[11];
  const double sf = sin(phi), cf = cos(phi);
  const double st = sin(th), ct = cos(th);
  const double sp = sin(psi), cp = cos(psi);
  const double T = u[0];
  dx[0] = x[6]; dx[1] = x[7]; dx[2] = x[8];
  dx[3] = P + (Q * sf + Rr * cf) * (st / ct);
  dx[4] = Q * cf - Rr * sf;
  dx[5] = (Q * sf + Rr * cf) / ct;
  dx[6] = (T / mass) * (cf * st * cp + sf * sp);
  dx[7] = (T / mass) * (cf * st * sp - sf * cp);
  dx[8] = (T / mass) * (cf * ct) - g;
  dx[9] = ((Iyy - Izz) * Q * Rr + u[1]) / Ixx;
  dx[10] = ((Izz - Ixx) * P * Rr + u[2]) / Iyy;
  dx[11] = ((Ixx - Iyy) * P * Q + u[3]) / Izz;
}

static int state_dim(int dyn) { return dyn == KPO_DI6 ? 6 : 12; }
static int ctrl_dim(int dyn) { return dyn == KPO_DI6 ? 3 : 4; }

/* One integration step of PropagateODE (eq. 2): explicit Euler or classic RK4
 * with the control held constant over the segment. */
void kpo_step(const kpo_problem* pb, const double* x, const double* u, double* xn) {
  const int n = state_dim(pb->dyn);
  const double h = pb->h;
  double k1[12], k2[12], k3[12], k4[12], t[12];
  kpo_deriv(pb, x, u, k1);
  if (pb->integ == KPO_EULER) {
    for (int i = 0; i < n; ++i) xn[i] = x[i] + h * k1[i];
    return;
  }
  for (int i = 0; i < n; ++i) t[i] = x[i] + 0.5 * h * k1[i];
  kpo_deriv(pb, t, u, k2);
  for (int i = 0; i < n; ++i) t[i] = x[i] + 0.5 * h * k2[i];
  kpo_deriv(pb, t, u, k3);
  for (int i = 0; i < n; ++i) t[i] = x[i] + h * k3[i];
  kpo_deriv(pb, t, u, k4);
  for (int i = 0; i < n; ++i) xn[i] = x[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* ------------------------------------------------------------------------ */
/* Validity (Alg. 2, "the trajectory from x to x' is valid").                */
/* ------------------------------------------------------------------------ */
/* State constraint: finite and inside the box, the box grown by `relax`
 * (relax < 0 shrinks it). */
int kpo_state_ok(const kpo_problem* pb, const double* x, double relax) {
  const int n = state_dim(pb->dyn);
  for (int i = 0; i < n; ++i) {
    if (!isfinite(x[i])) return 0;
    if (x[i] < pb->x_lo[i] - relax || x[i] > pb->x_hi[i] + relax) return 0;
  }
  return 1;
}

/* Collision: the axis-aligned box spanned by two consecutive positions,
 * grown by `inflate` on every side, against every closed obstacle box.
 * Touching counts as a hit.  (The paper's implementation bounds each dt
 * interval with a box and tests it against the obstacles.) */
int kpo_swept_hit(const kpo_problem* pb, const double* p0, const double* p1, double inflate) {
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = (p0[a] < p1[a] ? p0[a] : p1[a]) - inflate;
    hi[a] = (p0[a] < p1[a] ? p1[a] : p0[a]) + inflate;
  }
  for (int k = 0; k < pb->n_obs; ++k) {
    const double* o = pb->obs + 6 * k;
    int hit = 1;
    for (int a = 0; a < 3; ++a) {
      if (lo[a] > o[3 + a] || o[a] > hi[a]) { hit = 0; break; }
    }
    if (hit) return 1;
  }
  return 0;
}

/* First failing step of a stored trajectory traj[0..K] (traj[0] = parent):
 * step j fails if x_j leaves the (relaxed) state box or its swept box hits an
 * obstacle inflated by margin - relax.  Returns K + 1 if no step fails. */
static int first_fail(const kpo_problem* pb, const double* traj, int n, int K, double relax) {
  for (int j = 1; j <= K; ++j) {
    const double* xj = traj + (size_t)j * n;
    const double* xp = traj + (size_t)(j - 1) * n;
    if (!kpo_state_ok(pb, xj, relax)) return j;
    if (kpo_swept_hit(pb, xp, xj, pb->margin - relax)) return j;
  }
  return K + 1;
}

/* ------------------------------------------------------------------------ */
/* Decomposition: a uniform workspace grid of G regions per axis, each cut    */
/* into S sub-regions per axis.  Cell id = region * 64 + sub-cell index.      */
/* ------------------------------------------------------------------------ */
uint32_t kpo_cell_of(const kpo_problem* pb, const double* p) {
  int c[3];
  for (int a = 0; a < 3; ++a) {
    const int na = pb->grid[a] * pb->sub;
    const double t = (p[a] - pb->x_lo[a]) / (pb->x_hi[a] - pb->x_lo[a]) * (double)na;
    double fl = floor(t);
    if (fl < 0.0) fl = 0.0;
    if (fl > (double)(na - 1)) fl = (double)(na - 1);
    c[a] = (int)fl;
  }
  const int S = pb->sub;
  const uint32_t region = (uint32_t)(((c[2] / S) * pb->grid[1] + (c[1] / S)) * pb->grid[0] + (c[0] / S));
  const uint32_t local = (uint32_t)(((c[2] % S) * S + (c[1] % S)) * S + (c[0] % S));
  return region * 64u + local;
}

/* Whether position p lies within tol of an interior plane of the fine-cell
 * grid (a plane between two cells, not the clamped outer faces of W). */
int kpo_near_cell_plane(const kpo_problem* pb, const double* p, double tol) {
  for (int a = 0; a < 3; ++a) {
    const int na = pb->grid[a] * pb->sub;
    const double w = (pb->x_hi[a] - pb->x_lo[a]) / (double)na;
    const double t = (p[a] - pb->x_lo[a]) / w;
    const double k = floor(t + 0.5);
    if (k >= 1.0 && k <= (double)(na - 1) && fabs(t - k) * w < tol) return 1;
  }
  return 0;
}

static double goal_dist(const kpo_problem* pb, const double* p) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double d = p[a] - pb->goal_c[a];
    d2 += d * d;
  }
  return sqrt(d2);
}

/* ------------------------------------------------------------------------ */
/* Region estimates, Alg. 3 with eqs. (3)-(5).                               */
/* ------------------------------------------------------------------------ */
/* Score of one region.  With FreeVol = (delta + nv) vol / (delta + nv + ni)
 * (eq. 3) and Score = FreeVol^4 / ((1 + Cov)(1 + (nv + ni)^2)) (eq. 4), every
 * region of the uniform grid has the same vol, so vol^4 is a common factor of
 * every Score and cancels in the ratio of eq. (5); the score is kept without
 * it.  Fixed order of FP64 operations. */
double kpo_region_score(double delta, uint64_t nv, uint64_t ni, int cov) {
  const double a = delta + (double)nv;
  const double b = a + (double)ni;
  const double phi = a / b;
  const double phi2 = phi * phi;
  const double num = phi2 * phi2;
  const double n = (double)(nv + ni);
  const double den = (1.0 + (double)cov) * (1.0 + n * n);
  return num / den;
}

/* P_accept over R_avail (eq. 5): min(1, Score_i / sum_j Score_j + eps).
 * The sum is taken exactly: every score is scaled by the same power of two
 * 2^(46 - e), where 2^e <= max Score < 2^(e+1), and floored to an integer q_i
 * (so q_max lies in [2^46, 2^47)); Q = sum q_i is an exact integer sum and
 * P_i = min(1, q_i / Q + eps).  The threshold used by every "with probability
 * P" test is thr = floor(P * 2^32) (2^32 when P = 1): a uniform 32-bit word w
 * passes the test iff w < thr.  Regions outside R_avail keep P = 1. */
void kpo_estimates(int R, const uint8_t* avail, const uint64_t* nv, const uint64_t* ni,
                   const uint64_t* visited, double delta, double eps,
                   double* score_out, uint64_t* q_out, double* p_out, uint64_t* thr_out) {
  double smax = 0.0;
  for (int r = 0; r < R; ++r) {
    double s = 0.0;
    if (avail[r]) {
      int cov = __builtin_popcountll(visited[r]);
      s = kpo_region_score(delta, nv[r], ni[r], cov);
      if (s > smax) smax = s;
    }
    if (score_out) score_out[r] = s;
  }
  int e = 0;
  if (smax > 0.0) e = ilogb(smax);
  uint64_t Q = 0;
  for (int r = 0; r < R; ++r) {
    uint64_t q = 0;
    if (avail[r]) {
      int cov = __builtin_popcountll(visited[r]);
      double s = kpo_region_score(delta, nv[r], ni[r], cov);
      q = (uint64_t)floor(ldexp(s, 46 - e));
    }
    if (q_out) q_out[r] = q;
    Q += q;
  }
  for (int r = 0; r < R; ++r) {
    double P = 1.0;
    uint64_t thr = 4294967296ull;
    if (avail[r]) {
      int cov = __builtin_popcountll(visited[r]);
      double s = kpo_region_score(delta, nv[r], ni[r], cov);
      uint64_t q = (uint64_t)floor(ldexp(s, 46 - e));
      P = (Q > 0) ? (double)q / (double)Q + eps : eps;
      if (P >= 1.0) {
        P = 1.0;
      } else {
        thr = (uint64_t)floor(P * 4294967296.0);
      }
    }
    if (p_out) p_out[r] = P;
    if (thr_out) thr_out[r] = thr;
  }
}

/* ------------------------------------------------------------------------ */
/* Planner state.                                                            */
/* ------------------------------------------------------------------------ */
struct kpo_planner {
  kpo_problem pb;
  double* obs;
  int n, m, R, K;
  int32_t N, it, nF, lambda, nU, goal_id;
  uint64_t sum_lanes;
  double* x;
  float* u;
  int32_t* parent;
  uint32_t* cell;
  uint8_t* flag;
  int32_t* birth;
  int32_t* sample;
  uint64_t *nv, *ni, *visited, *thr;
  uint8_t* avail;
  int32_t* F;
  /* V_U: accepted samples not yet in the tree (Alg. 2 output) */
  int32_t* U_parent;
  int32_t* U_sample;
  double* U_x;
  float* U_u;
  uint32_t* U_cell;
  int32_t* U_goal;
};

static void* xcalloc(size_t n, size_t sz) {
  void* p = calloc(n ? n : 1, sz);
  return p;
}

static int alloc_arrays(kpo_planner* P) {
  const size_t cap = (size_t)P->pb.cap;
  P->x = xcalloc(cap * P->n, sizeof(double));
  P->u = xcalloc(cap * P->m, sizeof(float));
  P->parent = xcalloc(cap, sizeof(int32_t));
  P->cell = xcalloc(cap, sizeof(uint32_t));
  P->flag = xcalloc(cap, 1);
  P->birth = xcalloc(cap, sizeof(int32_t));
  P->sample = xcalloc(cap, sizeof(int32_t));
  P->nv = xcalloc(P->R, sizeof(uint64_t));
  P->ni = xcalloc(P->R, sizeof(uint64_t));
  P->visited = xcalloc(P->R, sizeof(uint64_t));
  P->thr = xcalloc(P->R, sizeof(uint64_t));
  P->avail = xcalloc(P->R, 1);
  P->F = xcalloc(cap, sizeof(int32_t));
  P->U_parent = xcalloc(cap, sizeof(int32_t));
  P->U_sample = xcalloc(cap, sizeof(int32_t));
  P->U_x = xcalloc(cap * P->n, sizeof(double));
  P->U_u = xcalloc(cap * P->m, sizeof(float));
  P->U_cell = xcalloc(cap, sizeof(uint32_t));
  P->U_goal = xcalloc(cap, sizeof(int32_t));
  return P->x && P->u && P->parent && P->cell && P->flag && P->birth && P->sample && P->nv &&
         P->ni && P->visited && P->thr && P->avail && P->F && P->U_parent && P->U_sample &&
         P->U_x && P->U_u && P->U_cell && P->U_goal;
}

void kpo_destroy(kpo_planner* P) {
  if (!P) return;
  free(P->obs);
  free(P->x); free(P->u); free(P->parent); free(P->cell); free(P->flag); free(P->birth);
  free(P->sample); free(P->nv); free(P->ni); free(P->visited); free(P->thr); free(P->avail);
  free(P->F); free(P->U_parent); free(P->U_sample); free(P->U_x); free(P->U_u);
  free(P->U_cell); free(P->U_goal);
  free(P);
}

static int ball_box_dist_le(const double* c, double r, const double* o) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double d = 0.0;
    if (c[a] < o[a]) d = o[a] - c[a];
    else if (c[a] > o[3 + a]) d = c[a] - o[3 + a];
    d2 += d * d;
  }
  return d2 <= r * r;
}

/* Alg. 1 set-up: root = x_init in V_E, every P_accept = 1. */
kpo_planner* kpo_create(const kpo_problem* pb, int32_t* status) {
  *status = KPO_E_ARG;
  if (!pb || (pb->dyn != KPO_DI6 && pb->dyn != KPO_QUAD12)) return NULL;
  if (pb->integ != KPO_EULER && pb->integ != KPO_RK4) return NULL;
  if (pb->steps < 1 || !(pb->h > 0.0) || pb->cap < 1 || pb->lambda_max < 1) return NULL;
  if (pb->sub < 1 || pb->sub > 4 || pb->n_obs < 0 || (pb->n_obs > 0 && !pb->obs)) return NULL;
  for (int a = 0; a < 3; ++a)
    if (pb->grid[a] < 1 || !(pb->x_hi[a] > pb->x_lo[a])) return NULL;
  if ((long)pb->grid[0] * pb->grid[1] * pb->grid[2] > 65536) return NULL;
  kpo_planner* P = xcalloc(1, sizeof(kpo_planner));
  P->pb = *pb;
  P->obs = xcalloc((size_t)6 * (pb->n_obs ? pb->n_obs : 1), sizeof(double));
  if (pb->n_obs) memcpy(P->obs, pb->obs, sizeof(double) * 6 * pb->n_obs);
  P->pb.obs = P->obs;
  P->n = state_dim(pb->dyn);
  P->m = ctrl_dim(pb->dyn);
  P->K = pb->steps;
  P->R = pb->grid[0] * pb->grid[1] * pb->grid[2];
  if (!alloc_arrays(P)) { kpo_destroy(P); return NULL; }
  /* x_init must be valid: inside the state box and clear of every obstacle
   * (a zero-length swept box at x_init). */
  if (!kpo_state_ok(&P->pb, pb->x_init, 0.0) ||
      kpo_swept_hit(&P->pb, pb->x_init, pb->x_init, pb->margin)) {
    *status = KPO_E_START_INVALID;
    kpo_destroy(P);
    return NULL;
  }
  /* X_goal must lie in the valid set: the ball inside W, clear of obstacles. */
  for (int a = 0; a < 3; ++a) {
    if (pb->goal_c[a] - pb->goal_r < pb->x_lo[a] || pb->goal_c[a] + pb->goal_r > pb->x_hi[a] ||
        !(pb->goal_r >= 0.0)) {
      *status = KPO_E_GOAL_INVALID;
      kpo_destroy(P);
      return NULL;
    }
  }
  for (int k = 0; k < pb->n_obs; ++k) {
    if (ball_box_dist_le(pb->goal_c, pb->goal_r + pb->margin, P->obs + 6 * k)) {
      *status = KPO_E_GOAL_INVALID;
      kpo_destroy(P);
      return NULL;
    }
  }
  memcpy(P->x, pb->x_init, sizeof(double) * P->n);
  P->parent[0] = -1;
  P->birth[0] = -1;
  P->sample[0] = -1;
  P->cell[0] = kpo_cell_of(&P->pb, pb->x_init);
  P->flag[0] = 1;
  P->N = 1;
  P->it = 0;
  P->goal_id = -1;
  for (int r = 0; r < P->R; ++r) P->thr[r] = 4294967296ull;
  P->visited[P->cell[0] >> 6] |= 1ull << (P->cell[0] & 63u);
  P->avail[P->cell[0] >> 6] = 1;
  /* x_init already in X_goal: a path with no edges. */
  if (goal_dist(&P->pb, pb->x_init) <= pb->goal_r) P->goal_id = 0;
  *status = KPO_OK;
  return P;
}

kpo_planner* kpo_clone(const kpo_planner* Q) {
  int32_t st;
  kpo_problem pb = Q->pb;
  pb.obs = Q->obs;
  kpo_planner* P = kpo_create(&pb, &st);
  if (!P) return NULL;
  const size_t cap = (size_t)Q->pb.cap;
  memcpy(P->x, Q->x, cap * Q->n * sizeof(double));
  memcpy(P->u, Q->u, cap * Q->m * sizeof(float));
  memcpy(P->parent, Q->parent, cap * 4);
  memcpy(P->cell, Q->cell, cap * 4);
  memcpy(P->flag, Q->flag, cap);
  memcpy(P->birth, Q->birth, cap * 4);
  memcpy(P->sample, Q->sample, cap * 4);
  memcpy(P->nv, Q->nv, Q->R * 8);
  memcpy(P->ni, Q->ni, Q->R * 8);
  memcpy(P->visited, Q->visited, Q->R * 8);
  memcpy(P->thr, Q->thr, Q->R * 8);
  memcpy(P->avail, Q->avail, Q->R);
  memcpy(P->F, Q->F, cap * 4);
  memcpy(P->U_parent, Q->U_parent, cap * 4);
  memcpy(P->U_sample, Q->U_sample, cap * 4);
  memcpy(P->U_x, Q->U_x, cap * Q->n * sizeof(double));
  memcpy(P->U_u, Q->U_u, cap * Q->m * sizeof(float));
  memcpy(P->U_cell, Q->U_cell, cap * 4);
  memcpy(P->U_goal, Q->U_goal, cap * 4);
  P->N = Q->N; P->it = Q->it; P->nF = Q->nF; P->lambda = Q->lambda; P->nU = Q->nU;
  P->goal_id = Q->goal_id; P->sum_lanes = Q->sum_lanes;
  return P;
}

/* Frontier and branching factor for this iteration: V_E as the list of
 * frontier node ids in ascending order, and eq. (6). */
int32_t kpo_frontier(kpo_planner* P) {
  int32_t nF = 0;
  for (int32_t i = 0; i < P->N; ++i)
    if (P->flag[i]) P->F[nF++] = i;
  P->nF = nF;
  P->lambda = 0;
  if (nF == 0) return KPO_FRONTIER_EMPTY;
  int32_t lam = (P->pb.cap - P->N) / nF;
  if (lam > P->pb.lambda_max) lam = P->pb.lambda_max;
  P->lambda = lam;
  if (lam == 0) return KPO_TREE_FULL;
  return KPO_OK;
}

int64_t kpo_num_lanes(const kpo_planner* P) { return (int64_t)P->nF * P->lambda; }

/* Alg. 2, one thread's work, in its order: sample u (dt is the segment of K
 * steps), x' = PropagateODE(x, u, dt) over the whole segment, map x' to its
 * sub-region, then decide validity.  The validity test is taken step by
 * step along the integrated trajectory (every step's state and swept box);
 * it does not move x'.  A non-finite x' is mapped to its parent's cell. */
void kpo_expand_one(const kpo_planner* P, int32_t f, int32_t s, kpo_record* rec, double* traj_out) {
  kpo_expand_one_u(P, f, s, NULL, rec, traj_out);
}

/* Whether the FP64 value of a state is a stable reference for a
 * lower-precision computation of the same trajectory: finite, and for the
 * quadcopter a pitch away from the Euler-angle singularity at |theta| = pi/2,
 * where the rate matrix W(phi, theta) has 1 / cos(theta) entries and nearby
 * trajectories separate without bound.  Used only to classify decisions in
 * the parity protocol; it changes no planner result. */
static int well_conditioned(const kpo_problem* pb, const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  if (pb->dyn == KPO_QUAD12 && fabs(x[4]) > pb->cond_tilt) return 0;
  return 1;
}

/* The same expansion with the control given by the caller (u_given: m FP32
 * values; NULL draws it as above).  The acceptance word is drawn as above. */
void kpo_expand_one_u(const kpo_planner* P, int32_t f, int32_t s, const float* u_given,
                      kpo_record* rec, double* traj_out) {
  const kpo_problem* pb = &P->pb;
  const int n = P->n, m = P->m, K = P->K;
  double trajbuf[12 * 65];
  double* traj = traj_out;
  double* heap = NULL;
  if (!traj) {
    if ((size_t)(K + 1) * n <= sizeof(trajbuf) / sizeof(double)) traj = trajbuf;
    else traj = heap = malloc(sizeof(double) * (size_t)(K + 1) * n);
  }
  memset(rec, 0, sizeof(*rec));
  rec->parent = f;
  rec->sample = s;
  draw_expansion(pb, m, (uint32_t)P->it, (uint32_t)f, (uint32_t)s, rec->u, &rec->w_acc);
  if (u_given)
    for (int j = 0; j < m; ++j) rec->u[j] = u_given[j];
  const int Kl = kpo_segment_steps(pb, (uint32_t)P->it, (uint32_t)f, (uint32_t)s);
  rec->k_seg = Kl;
  double u[4] = {0, 0, 0, 0};
  for (int j = 0; j < m; ++j) u[j] = (double)rec->u[j];
  /* x' = PropagateODE(x, u, dt) */
  memcpy(traj, P->x + (size_t)f * n, sizeof(double) * n);
  for (int j = 1; j <= Kl; ++j) kpo_step(pb, traj + (size_t)(j - 1) * n, u, traj + (size_t)j * n);
  rec->steps = Kl;
  const double* xe = traj + (size_t)Kl * n;
  memcpy(rec->x, xe, sizeof(double) * n);
  /* map x' to its sub-region R_i^k */
  const double tol = pb->amb_tol;
  if (isfinite(xe[0]) && isfinite(xe[1]) && isfinite(xe[2])) {
    rec->cell = kpo_cell_of(pb, xe);
    rec->amb_cell = kpo_near_cell_plane(pb, xe, tol);
  } else {
    rec->cell = P->cell[f];
    rec->amb_cell = 0;
  }
  /* validity of the trajectory from x to x' */
  rec->fail = first_fail(pb, traj, n, Kl, 0.0);
  rec->fail_strict = first_fail(pb, traj, n, Kl, -tol);
  rec->fail_loose = first_fail(pb, traj, n, Kl, +tol);
  rec->valid = (rec->fail == Kl + 1);
  rec->cond_step = Kl + 1;
  for (int j = 1; j <= Kl; ++j) {
    if (!well_conditioned(pb, traj + (size_t)j * n, n)) {
      rec->cond_step = j;
      break;
    }
  }
  const double gd = goal_dist(pb, xe);
  rec->goal = rec->valid && gd <= pb->goal_r;
  rec->amb_goal = fabs(gd - pb->goal_r) < tol;
  free(heap);
}

/* Every lane of Alg. 2, lane k = (frontier position e, sample s) with
 * k = e * lambda + s.  Lanes are independent of each other (each reads only
 * the tree as it was when the iteration started), so with OpenMP they may
 * run on several threads; every record is the same either way. */
int64_t kpo_expand_all(const kpo_planner* P, kpo_record* recs) {
  return kpo_expand_all_u(P, NULL, recs);
}

/* All lanes with given controls: U holds 4 floats per lane, lane order
 * (NULL: the controls are drawn). */
int64_t kpo_expand_all_u(const kpo_planner* P, const float* U, kpo_record* recs) {
  const int64_t lanes = (int64_t)P->nF * P->lambda;
  const int32_t lam = P->lambda;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) if (lanes > 256)
#endif
  for (int64_t k = 0; k < lanes; ++k) {
    const int32_t e = (int32_t)(k / lam), s = (int32_t)(k - (int64_t)e * lam);
    kpo_expand_one_u(P, P->F[e], s, U ? U + 4 * k : NULL, &recs[k], NULL);
  }
  return lanes;
}

void kpo_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int32_t kpo_get_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* Alg. 2 bookkeeping, in lane order (frontier order, then sample index):
 * valid -> n_valid(R_i)++ and accept if the sub-region is unvisited or the
 * acceptance word passes P_accept(R_i); invalid -> n_invalid(R_i)++.
 * "Unvisited" refers to the tree as it was when the iteration started. */
void kpo_apply(kpo_planner* P, const kpo_record* recs, int64_t nrec) {
  const int n = P->n, m = P->m;
  P->nU = 0;
  for (int64_t k = 0; k < nrec; ++k) {
    const kpo_record* r = &recs[k];
    const uint32_t reg = r->cell >> 6;
    if (r->valid) {
      P->nv[reg] += 1;
      const int unvisited = !((P->visited[reg] >> (r->cell & 63u)) & 1ull);
      const int accept = unvisited || ((uint64_t)r->w_acc < P->thr[reg]);
      if (accept) {
        const int32_t j = P->nU++;
        P->U_parent[j] = r->parent;
        P->U_sample[j] = r->sample;
        memcpy(P->U_x + (size_t)j * n, r->x, sizeof(double) * n);
        memcpy(P->U_u + (size_t)j * m, r->u, sizeof(float) * m);
        P->U_cell[j] = r->cell;
        P->U_goal[j] = r->goal;
      }
    } else {
      P->ni[reg] += 1;
    }
  }
  P->sum_lanes += (uint64_t)nrec;
}

/* Alg. 3.  R_avail = regions holding a node of the tree; V_U is not in the
 * tree yet at this point of the iteration. */
void kpo_update_estimates(kpo_planner* P) {
  kpo_estimates(P->R, P->avail, P->nv, P->ni, P->visited, P->pb.delta, P->pb.eps, NULL, NULL,
                NULL, P->thr);
}

/* Two node-set words for node i in iteration it: one Philox block serves the
 * node pair (2k, 2k+1) through counter (it, k, 0, 3); node 2k takes words 0
 * and 1, node 2k+1 words 2 and 3.  The first word of the pair decides the
 * move V_E -> V_O, the second the move V_O -> V_E. */
static void node_words(const kpo_planner* P, int32_t i, uint32_t* w_dem, uint32_t* w_pro) {
  uint32_t key[2] = {(uint32_t)P->pb.seed, (uint32_t)(P->pb.seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)P->it, (uint32_t)i >> 1, 0u, 3u};
  uint32_t w[4];
  kpo_philox4x32_10(ctr, key, w);
  *w_dem = w[2 * (i & 1)];
  *w_pro = w[2 * (i & 1) + 1];
}

/* Alg. 4, in its order.  First, each x in V_E moves to V_O with probability
 * 1 - P_accept (w_dem >= thr).  Then V_U joins V_E and the tree in lane
 * order; the first new node in X_goal ends the run (its id is returned) and
 * the last step is not reached.  Last, each x in V_O, including the ones
 * just moved there, returns to V_E with probability P_accept (w_pro < thr). */
int32_t kpo_update_node_sets(kpo_planner* P) {
  const int n = P->n, m = P->m;
  const int32_t N0 = P->N;
  for (int32_t i = 0; i < N0; ++i) {
    if (!P->flag[i]) continue;
    uint32_t wd, wp;
    node_words(P, i, &wd, &wp);
    if ((uint64_t)wd >= P->thr[P->cell[i] >> 6]) P->flag[i] = 0;
  }
  int32_t goal = -1;
  for (int32_t k = 0; k < P->nU; ++k) {
    const int32_t id = N0 + k;
    memcpy(P->x + (size_t)id * n, P->U_x + (size_t)k * n, sizeof(double) * n);
    memcpy(P->u + (size_t)id * m, P->U_u + (size_t)k * m, sizeof(float) * m);
    P->parent[id] = P->U_parent[k];
    P->sample[id] = P->U_sample[k];
    P->birth[id] = P->it;
    P->cell[id] = P->U_cell[k];
    P->flag[id] = 1;
    P->visited[P->U_cell[k] >> 6] |= 1ull << (P->U_cell[k] & 63u);
    P->avail[P->U_cell[k] >> 6] = 1;
    if (goal < 0 && P->U_goal[k]) goal = id;
  }
  P->N = N0 + P->nU;
  P->nU = 0;
  if (goal < 0) {
    for (int32_t i = 0; i < N0; ++i) {
      if (P->flag[i]) continue;
      uint32_t wd, wp;
      node_words(P, i, &wd, &wp);
      if ((uint64_t)wp < P->thr[P->cell[i] >> 6]) P->flag[i] = 1;
    }
  }
  P->it += 1;
  if (goal >= 0) P->goal_id = goal;
  return goal;
}

int32_t kpo_iterate(kpo_planner* P, int32_t* goal_id) {
  *goal_id = -1;
  if (P->goal_id >= 0) { *goal_id = P->goal_id; return KPO_SOLVED; }
  int32_t st = kpo_frontier(P);
  if (st != KPO_OK) return st;
  const int64_t lanes = kpo_num_lanes(P);
  kpo_record* recs = malloc(sizeof(kpo_record) * (size_t)(lanes ? lanes : 1));
  kpo_expand_all(P, recs);
  kpo_apply(P, recs, lanes);
  free(recs);
  kpo_update_estimates(P);
  int32_t g = kpo_update_node_sets(P);
  if (g >= 0) { *goal_id = g; return KPO_SOLVED; }
  return KPO_OK;
}

static double now_ms(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

/* Alg. 1's loop: until a goal node appears, the frontier empties,
 * the tree is full, or the iteration / wall-clock budget runs out. */
int32_t kpo_plan(kpo_planner* P, int32_t max_iters, double t_max_ms, int32_t* goal_id,
                 int32_t* iters) {
  const double t0 = now_ms();
  *iters = 0;
  *goal_id = -1;
  if (P->goal_id >= 0) { *goal_id = P->goal_id; return KPO_SOLVED; }
  while (*iters < max_iters && now_ms() - t0 < t_max_ms) {
    int32_t st = kpo_iterate(P, goal_id);
    *iters += 1;
    if (st != KPO_OK) return st;
  }
  return KPO_TIMEOUT;
}

/* "Return trajectory x_init to x": node ids from the root to `node`. */
int32_t kpo_path(const kpo_planner* P, int32_t node, int32_t* ids, int32_t cap) {
  int32_t len = 0;
  for (int32_t v = node; v >= 0; v = P->parent[v]) len++;
  if (len > cap) return -len;
  int32_t k = len;
  for (int32_t v = node; v >= 0; v = P->parent[v]) ids[--k] = v;
  return len;
}

int32_t kpo_replay(const kpo_problem* pb, const double* x0, int32_t n_edges, const float* controls,
                   double margin, double* end_states, int32_t* reached_goal) {
  return kpo_replay_k(pb, x0, n_edges, controls, NULL, margin, end_states, reached_goal);
}

int32_t kpo_replay_k(const kpo_problem* pb, const double* x0, int32_t n_edges, const float* controls,
                     const int32_t* edge_steps, double margin, double* end_states,
                     int32_t* reached_goal) {
  const int n = state_dim(pb->dyn), m = ctrl_dim(pb->dyn);
  kpo_problem q = *pb;
  q.margin = margin;
  double x[12], xn[12], u[4] = {0, 0, 0, 0};
  memcpy(x, x0, sizeof(double) * n);
  int valid = kpo_state_ok(&q, x, 0.0) && !kpo_swept_hit(&q, x, x, margin);
  for (int32_t e = 0; e < n_edges; ++e) {
    for (int j = 0; j < m; ++j) u[j] = (double)controls[(size_t)e * m + j];
    const int ke = edge_steps ? edge_steps[e] : pb->steps;
    for (int k = 0; k < ke; ++k) {
      kpo_step(&q, x, u, xn);
      if (!kpo_state_ok(&q, xn, 0.0) || kpo_swept_hit(&q, x, xn, margin)) valid = 0;
      memcpy(x, xn, sizeof(double) * n);
    }
    if (end_states) memcpy(end_states + (size_t)e * n, x, sizeof(double) * n);
  }
  *reached_goal = goal_dist(pb, x) <= pb->goal_r;
  return valid;
}

/* FP64 replay of a stored trajectory one edge at a time.  Edge e starts
 * from its parent's stored state xs[e] (n FP32 values, widened), holds the
 * stored control us[e] for steps[e] steps, and must keep every step inside
 * the state box relaxed by tol and every swept box clear of the obstacles
 * grown by margin - tol (margin 0 replays against the obstacles themselves);
 * its end is compared with the stored child xs[e + 1].  A replay from the
 * root alone would compound the FP32 rounding of the stored states along the
 * path (the quadcopter is open-loop unstable), so each edge is checked from
 * the state the planner integrated it from.  Returns 1 if every edge is
 * valid; *worst gets the largest |end - child| / max(1, |end|) over all
 * components, *first_bad the first invalid edge (-1: none), and end the FP64
 * end state of the last edge. */
int32_t kpo_replay_edges(const kpo_problem* pb, int32_t n_edges, const float* xs, const float* us,
                         const int32_t* steps, double margin, double tol, double* worst,
                         int32_t* first_bad, double* end) {
  const int n = state_dim(pb->dyn), m = ctrl_dim(pb->dyn);
  kpo_problem q = *pb;
  q.margin = margin;
  double x[12], xn[12], u[4] = {0, 0, 0, 0};
  *worst = 0.0;
  *first_bad = -1;
  for (int i = 0; i < n; ++i) x[i] = (double)xs[i];
  for (int32_t e = 0; e < n_edges; ++e) {
    for (int i = 0; i < n; ++i) x[i] = (double)xs[(size_t)e * n + i];
    for (int j = 0; j < m; ++j) u[j] = (double)us[(size_t)(e + 1) * m + j];
    int ok = 1;
    for (int k = 0; k < steps[e + 1]; ++k) {
      kpo_step(&q, x, u, xn);
      if (!kpo_state_ok(&q, xn, tol) || kpo_swept_hit(&q, x, xn, margin - tol)) ok = 0;
      memcpy(x, xn, sizeof(double) * n);
    }
    if (!ok && *first_bad < 0) *first_bad = e;
    for (int i = 0; i < n; ++i) {
      const double ref = fabs(x[i]) > 1.0 ? fabs(x[i]) : 1.0;
      const double d = fabs((double)xs[(size_t)(e + 1) * n + i] - x[i]) / ref;
      if (!(d <= *worst)) *worst = d;  /* NaN propagates */
    }
  }
  if (end) memcpy(end, x, sizeof(double) * n);
  return *first_bad < 0;
}

/* Integrate n_seg segments in FP64: segment i starts at x0[i] (n values),
 * holds control u[i] (m FP32 values) and runs steps[i] integration steps;
 * the end state goes to out[i].  A plain primitive used to re-check edges. */
void kpo_integrate_batch(const kpo_problem* pb, int64_t n_seg, const double* x0, const float* u,
                         const int32_t* steps, double* out) {
  const int n = state_dim(pb->dyn), m = ctrl_dim(pb->dyn);
  for (int64_t i = 0; i < n_seg; ++i) {
    double x[12], xn[12], uu[4] = {0, 0, 0, 0};
    memcpy(x, x0 + (size_t)i * n, sizeof(double) * n);
    for (int j = 0; j < m; ++j) uu[j] = (double)u[(size_t)i * m + j];
    for (int k = 0; k < steps[i]; ++k) {
      kpo_step(pb, x, uu, xn);
      memcpy(x, xn, sizeof(double) * n);
    }
    memcpy(out + (size_t)i * n, x, sizeof(double) * n);
  }
}

void kpo_get_view(kpo_planner* P, kpo_view* v) {
  v->n = P->n; v->m = P->m; v->R = P->R; v->cap = P->pb.cap;
  v->N = P->N; v->it = P->it; v->nF = P->nF; v->lambda = P->lambda; v->nU = P->nU;
  v->goal_id = P->goal_id;
  v->x = P->x; v->u = P->u; v->parent = P->parent; v->cell = P->cell; v->flag = P->flag;
  v->birth = P->birth; v->sample = P->sample; v->nv = P->nv; v->ni = P->ni;
  v->visited = P->visited; v->avail = P->avail; v->thr = P->thr; v->F = P->F;
  v->sum_lanes = P->sum_lanes;
}

void kpo_set_counters(kpo_planner* P, int32_t N, int32_t it) {
  P->N = N;
  P->it = it;
}

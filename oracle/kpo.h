/*
 * Kino-PAX CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential FP64 implementation of one Kino-PAX planning run
 * (Perrault, Ho, Lahijanian, "Kino-PAX: Highly Parallel Kinodynamic
 * Sampling-based Planner", RA-L 2025): Alg. 1 (main loop), Alg. 2
 * (Propagate), Alg. 3 (UpdateEstimates, eqs. 3-5), Alg. 4 (UpdateNodeSets)
 * and eq. 6 (branching factor).  It shares no code, header or constant table
 * with the GPU library; only the tests, the smoke check and the bench's CPU
 * baseline may load it.  Product code must never call it.
 *
 * Precision: dynamics, validity, cell and goal tests in FP64.  Sampled
 * controls are FP32 numbers (each is the FP32 value of a fixed map of one
 * Philox word, then widened exactly).  Region scores in FP64, their sum as an
 * exact integer (see kpo_update_estimates).  Counts, sets and ids exact.
 */
#ifndef KPO_H
#define KPO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { KPO_DI6 = 0, KPO_QUAD12 = 1 };
enum { KPO_EULER = 0, KPO_RK4 = 1 };
enum {
  KPO_OK = 0, KPO_SOLVED = 1, KPO_TIMEOUT = 2, KPO_TREE_FULL = 3,
  KPO_FRONTIER_EMPTY = 4, KPO_E_ARG = -1, KPO_E_START_INVALID = -4,
  KPO_E_GOAL_INVALID = -5
};

typedef struct {
  int32_t dyn;          /* KPO_DI6 or KPO_QUAD12 */
  int32_t integ;        /* KPO_EULER or KPO_RK4 */
  int32_t steps;        /* integration steps per segment */
  int32_t n_obs;
  double h;             /* step size */
  double prm[8];        /* quadcopter: mass, gravity, Ixx, Iyy, Izz */
  float u_lo[4], u_hi[4];
  double x_lo[12], x_hi[12];
  const double* obs;    /* [n_obs][6] lo xyz, hi xyz; copied at create */
  double margin;
  double x_init[12];
  double goal_c[3];
  double goal_r;
  int32_t grid[3];
  int32_t sub;          /* sub-regions per region axis, 1..4 */
  int32_t cap;          /* t_e */
  int32_t lambda_max;
  double delta, eps;
  uint64_t seed;
  double amb_tol;       /* ambiguity band for decisions taken on FP values */
  int32_t dur_mode;     /* 0: every segment takes `steps` steps; 1: k ~ U{1..steps} per expansion */
  int32_t pad_;
  double cond_tilt;     /* quadcopter: |pitch| above this marks a trajectory as ill-conditioned */
} kpo_problem;

/* One expansion (parent f, sample s) of Alg. 2, before any bookkeeping. */
typedef struct {
  int32_t parent;
  int32_t sample;
  float u[4];           /* sampled control (FP32 values) */
  double x[12];         /* x' = PropagateODE(x, u, dt): the end of the segment */
  int32_t steps;        /* steps integrated to reach x' (the segment's steps) */
  int32_t valid;        /* segment valid */
  uint32_t cell;        /* fine cell of x' (region << 6 | sub-cell) */
  int32_t goal;         /* valid and x' in X_goal */
  uint32_t w_acc;       /* Philox word for the acceptance test */
  int32_t fail_strict;  /* first failing step with every test tightened by amb_tol (K+1: none) */
  int32_t fail_loose;   /* first failing step with every test relaxed by amb_tol */
  int32_t amb_cell;     /* x' within amb_tol of an interior cell plane */
  int32_t amb_goal;     /* x' within amb_tol of the goal sphere */
  int32_t k_seg;        /* integration steps of this segment (its duration / h) */
  int32_t fail;         /* first failing step (k_seg + 1: the segment is valid) */
  int32_t cond_step;    /* first step whose state is ill-conditioned (k_seg + 1: none) */
} kpo_record;

typedef struct kpo_planner kpo_planner;

/* --- primitives (exposed for the pins) --- */
void kpo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float kpo_control_map(uint32_t w, float lo, float hi);
void kpo_deriv(const kpo_problem* pb, const double* x, const double* u, double* dx);
void kpo_step(const kpo_problem* pb, const double* x, const double* u, double* xn);
int kpo_state_ok(const kpo_problem* pb, const double* x, double relax);
int kpo_swept_hit(const kpo_problem* pb, const double* p0, const double* p1, double inflate);
uint32_t kpo_cell_of(const kpo_problem* pb, const double* p);
int kpo_near_cell_plane(const kpo_problem* pb, const double* p, double tol);
double kpo_region_score(double delta, uint64_t nv, uint64_t ni, int cov);
void kpo_estimates(int R, const uint8_t* avail, const uint64_t* nv, const uint64_t* ni,
                   const uint64_t* visited, double delta, double eps,
                   double* score_out, uint64_t* q_out, double* p_out, uint64_t* thr_out);

/* Steps of the segment of expansion (it, f, s): `steps` when dur_mode = 0,
 * else 1 + floor(w * steps / 2^32) for word 1 of Philox(it, f, s, 1). */
int32_t kpo_segment_steps(const kpo_problem* pb, uint32_t it, uint32_t f, uint32_t s);

/* --- planner --- */
kpo_planner* kpo_create(const kpo_problem* pb, int32_t* status);
kpo_planner* kpo_clone(const kpo_planner* P);
void kpo_destroy(kpo_planner* P);
int32_t kpo_frontier(kpo_planner* P);                          /* eq. 6 + frontier list */
int64_t kpo_num_lanes(const kpo_planner* P);                   /* |V_E| * lambda */
void kpo_expand_one(const kpo_planner* P, int32_t f, int32_t s, kpo_record* rec, double* traj);
int64_t kpo_expand_all(const kpo_planner* P, kpo_record* recs); /* Alg. 2, per-lane part */
void kpo_expand_one_u(const kpo_planner* P, int32_t f, int32_t s, const float* u_given,
                      kpo_record* rec, double* traj);               /* given control */
int64_t kpo_expand_all_u(const kpo_planner* P, const float* U, kpo_record* recs);
/* Threads of the expansion loop (OpenMP builds; results do not depend on it). */
void kpo_set_threads(int32_t n);
int32_t kpo_get_threads(void);
void kpo_apply(kpo_planner* P, const kpo_record* recs, int64_t n); /* Alg. 2 bookkeeping */
void kpo_update_estimates(kpo_planner* P);                     /* Alg. 3 */
int32_t kpo_update_node_sets(kpo_planner* P);                  /* Alg. 4; goal id or -1 */
int32_t kpo_iterate(kpo_planner* P, int32_t* goal_id);         /* one pass of Alg. 1's loop */
int32_t kpo_plan(kpo_planner* P, int32_t max_iters, double t_max_ms, int32_t* goal_id,
                 int32_t* iters);
int32_t kpo_path(const kpo_planner* P, int32_t node, int32_t* ids, int32_t cap);

/* FP64 replay of a path: integrate from x0 under the given controls (n_edges x m),
 * check every step against the state box and the obstacles inflated by `margin`,
 * and test the goal at the end.  Writes the FP64 end state of every edge. */
int32_t kpo_replay(const kpo_problem* pb, const double* x0, int32_t n_edges, const float* controls,
                   double margin, double* end_states, int32_t* reached_goal);
/* The same with edge_steps[e] integration steps for edge e (NULL: `steps`). */
int32_t kpo_replay_k(const kpo_problem* pb, const double* x0, int32_t n_edges, const float* controls,
                     const int32_t* edge_steps, double margin, double* end_states,
                     int32_t* reached_goal);

/* Edge-by-edge FP64 replay of a stored trajectory of n_edges + 1 nodes:
 * xs [n_edges + 1][n] states, us [n_edges + 1][m] controls of the edge into
 * each node (row 0 unused), steps [n_edges + 1] steps of that edge. */
int32_t kpo_replay_edges(const kpo_problem* pb, int32_t n_edges, const float* xs, const float* us,
                         const int32_t* steps, double margin, double tol, double* worst,
                         int32_t* first_bad, double* end);

void kpo_integrate_batch(const kpo_problem* pb, int64_t n_seg, const double* x0, const float* u,
                         const int32_t* steps, double* out);

/* --- state access (arrays owned by the planner) --- */
typedef struct {
  int32_t n, m, R, cap;
  int32_t N, it, nF, lambda, nU, goal_id;
  double* x;           /* [cap][n] */
  float* u;            /* [cap][m] */
  int32_t* parent;
  uint32_t* cell;
  uint8_t* flag;       /* 1 = V_E, 0 = V_O */
  int32_t* birth;      /* iteration that created the node (-1 for the root) */
  int32_t* sample;     /* sample index of the creating expansion (-1 for the root) */
  uint64_t* nv;
  uint64_t* ni;
  uint64_t* visited;   /* [R], bit k = sub-cell k visited */
  uint8_t* avail;      /* region holds a tree node */
  uint64_t* thr;       /* acceptance threshold, P_accept * 2^32 */
  int32_t* F;          /* frontier list */
  uint64_t sum_lanes;  /* sum over iterations of |V_E| * lambda */
} kpo_view;
void kpo_get_view(kpo_planner* P, kpo_view* v);
void kpo_set_counters(kpo_planner* P, int32_t N, int32_t it);

#ifdef __cplusplus
}
#endif
#endif

/*
 * kp.h -- C ABI of the MI355X (gfx950) Kino-PAX tree-growth library.
 *
 * Kino-PAX (Perrault, Ho, Lahijanian, RA-L 2025) grows one tree of trajectory
 * segments.  Each iteration of its main loop (Alg. 1) runs three parallel
 * subroutines: Propagate (Alg. 2), UpdateEstimates (Alg. 3, eqs. 3-5) and
 * UpdateNodeSets (Alg. 4); the branching factor follows eq. (6).  This
 * library runs that loop on one GPU with hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Plain C types only.  Host pointers are read during the call and never
 *     kept, except where stated.  Device pointers are borrowed.
 *   - The caller allocates all device memory: one workspace buffer of
 *     kp_workspace_bytes() bytes (256-byte aligned) per problem.  The library
 *     allocates no device memory of its own.
 *   - All device work is enqueued on the HIP stream given at creation
 *     (hipStream_t passed as void*; NULL means the default stream).
 *   - Return value < 0 is an error; kp_last_error() then holds a message.
 *     Arguments are checked before any device work is enqueued.  No C++
 *     exception crosses this boundary.
 *   - A handle is not thread-safe: use one handle per host thread / stream.
 */
#ifndef KP_H
#define KP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KP_ABI_VERSION 3u
#define KP_MAX_STATE 12
#define KP_MAX_CONTROL 4
#define KP_MAX_OBSTACLES 2048  /* the obstacle table and candidate lists of a propagate block fit
                                   gfx950's LDS (69 KB per 256-lane block at 2048) */

typedef enum {
  KP_OK = 0,
  KP_SOLVED = 1,          /* a new tree node reached X_goal (goal test of Alg. 4) */
  KP_TIMEOUT = 2,         /* t_max or max_iters reached (loop bound of Alg. 1) */
  KP_TREE_FULL = 3,       /* eq. (6) gave lambda = 0: |T| + |V_E| > t_e */
  KP_FRONTIER_EMPTY = 4,  /* V_E became empty */
  KP_E_ARG = -1,          /* invalid argument (null pointer, bad size, bad field) */
  KP_E_DEVICE = -2,       /* a HIP call failed or a kernel reported an error */
  KP_E_WORKSPACE = -3,    /* workspace too small or misaligned */
  KP_E_START_INVALID = -4,/* x_init outside X_valid (Problem 1 requires x_init in X_valid) */
  KP_E_GOAL_INVALID = -5, /* X_goal not inside X_valid (Problem 1 requires it) */
  KP_E_ORDER = -6         /* calls made out of the Alg. 1 order */
} kp_status;

enum { KP_DYN_DI6 = 0, KP_DYN_QUAD12 = 1 };   /* 6D double integrator, 12D quadcopter */
enum { KP_INT_EULER = 0, KP_INT_RK4 = 1 };     /* explicit Euler, classic RK4 */

/*
 * Problem 1 plus the planner's hyperparameters.  All values are copied at
 * kp_create_problem(); the obstacle array is copied too.
 *
 * Dynamics (eq. 1).  KP_DYN_DI6: state (px py pz vx vy vz), control (ax ay az).
 * KP_DYN_QUAD12: state (px py pz, phi theta psi, vx vy vz, p q r), control
 * (thrust, tau_x, tau_y, tau_z); dyn_params = (mass, gravity, Ixx, Iyy, Izz).
 * A segment integrates `steps` steps of size `h` under one control (eq. 2).
 *
 * X_valid: x_lo <= x <= x_hi componentwise (closed), and every swept box of
 * two consecutive positions, grown by `margin`, clear of every obstacle.  The
 * first three state components are positions; x_lo[0..2], x_hi[0..2] is the
 * workspace W.  Obstacles are closed boxes, n_obstacles x 6 floats
 * (lo x, lo y, lo z, hi x, hi y, hi z), row-major.
 *
 * X_goal: the closed ball of goal_radius around goal_center (positions).
 *
 * Decomposition R (Sec. III-A.1): grid[0] x grid[1] x grid[2] regions over W,
 * each split into sub^3 sub-regions (1 <= sub <= 4).
 *
 * node_cap is t_e (Sec. IV-A), lambda_max the cap in eq. (6); delta (eq. 3)
 * and epsilon (eq. 5) are the constants of the region score and acceptance
 * probability.  seed keys the counter-based random generator.  t_max_ms is
 * Alg. 1's time budget for kp_plan; max_iters bounds the iterations too.
 * iters_per_sync: iterations kp_plan enqueues between two reads of the
 * device status word (0 = library default); results do not depend on it.
 */
typedef struct {
  uint32_t abi_version;        /* must be KP_ABI_VERSION */
  int32_t dynamics;            /* KP_DYN_* */
  int32_t integrator;          /* KP_INT_* */
  int32_t steps;               /* >= 1 */
  float h;                     /* > 0 */
  float dyn_params[8];
  float u_lo[KP_MAX_CONTROL], u_hi[KP_MAX_CONTROL];
  float x_lo[KP_MAX_STATE], x_hi[KP_MAX_STATE];
  const float* obstacles;      /* host pointer, n_obstacles * 6 floats */
  int32_t n_obstacles;         /* 0 .. KP_MAX_OBSTACLES */
  float margin;                /* >= 0 */
  float x_init[KP_MAX_STATE];
  float goal_center[3];
  float goal_radius;
  int32_t grid[3];             /* regions per axis, product <= 65536 */
  int32_t sub;                 /* 1..4 */
  int32_t node_cap;            /* t_e, 1 .. 2^30 */
  int32_t lambda_max;          /* 1 .. 255 */
  double delta;                /* > 0 */
  double epsilon;              /* in (0, 1] */
  uint64_t seed;
  double t_max_ms;
  int32_t max_iters;
  int32_t iters_per_sync;
  int32_t duration_mode;       /* 0: every segment is `steps` steps (default); 1: Alg. 2's random
                                  duration, k uniform in 1..steps steps per expansion, from word 1
                                  of Philox(it, parent, sample, 1) as 1 + (w * steps >> 32) */
  int32_t reserved;            /* must be 0 */
} kp_problem_desc;

typedef struct kp_problem kp_problem;

/* Result of kp_plan. */
typedef struct {
  int32_t status;          /* KP_SOLVED, KP_TIMEOUT, KP_TREE_FULL, KP_FRONTIER_EMPTY */
  int32_t goal_id;         /* tree node in X_goal, or -1 */
  int32_t iterations;      /* iterations of Alg. 1's loop executed */
  int32_t n_nodes;         /* |T| at the end */
  int32_t path_len;        /* nodes on the root-to-goal path (0 if none) */
  int32_t pad;
  double elapsed_ms;       /* wall clock of the loop, host side */
  uint64_t lanes_total;    /* expansions attempted: sum of |V_E| * lambda */
  uint64_t valid_total;    /* valid expansions: sum of n_valid increments */
} kp_plan_result;

/* Device counters after the last completed call (synchronises the stream). */
typedef struct {
  int32_t n_nodes;         /* |T| */
  int32_t n_frontier;      /* |V_E| for the next expansion */
  int32_t lambda;          /* eq. (6) for the next expansion */
  int32_t iteration;       /* iterations completed */
  int32_t goal_id;         /* -1 if none */
  int32_t done_code;       /* 0 while running, else a kp_status > 0 */
  int32_t n_new;           /* |V_U| of the last expansion */
  int32_t device_error;    /* nonzero if a kernel hit an internal limit */
  uint64_t lanes_total, valid_total, invalid_total;
  uint64_t steps_total;    /* integration steps executed (every lane runs its whole segment) */
  uint64_t box_tests_total;/* swept-box vs obstacle tests executed */
  uint64_t checked_steps_total; /* steps whose state and swept box were tested: each lane
                                   tests up to and including its first failing step */
  int32_t grid_propagate;  /* workgroups of a full-size propagate launch */
  int32_t grid_nodes;      /* workgroups of a full-size node-pass launch */
} kp_iter_stats;

/*
 * Host copy of the planner state (kp_copy_tree / kp_load_tree).  The caller
 * owns every buffer.  Node arrays are structure-of-arrays with n_nodes
 * columns: x is [n][n_nodes] floats (n = 6 or 12), u is [m][n_nodes] floats
 * (m = 3 or 4; the control of the edge into each node, zero for the root).
 * cell = region * 64 + sub-region index; flag 1 = V_E, 0 = V_O; birth = the
 * iteration that created the node (-1 for the root); sample = the expansion
 * index of that node's creation (0 for the root).  Region arrays have
 * R = grid[0]*grid[1]*grid[2] entries: visited has bit k set when sub-region
 * k of the region holds a tree node; thr is P_accept * 2^32 (2^32 for P = 1).
 */
typedef struct {
  int32_t n_nodes;
  int32_t iteration;
  float* x;
  float* u;
  int32_t* parent;
  uint32_t* cell;
  uint8_t* flag;
  int32_t* birth;
  uint8_t* sample;
  uint64_t* nv;
  uint64_t* ni;
  uint64_t* visited;
  uint8_t* avail;
  uint64_t* thr;
} kp_tree_host;

/*
 * One record per expansion lane of kp_expand, written when a trace buffer is
 * passed (lane = frontier position * lambda + sample).  100 bytes, device
 * memory of at least kp_trace_bytes() bytes.
 */
typedef struct {
  int32_t parent;          /* tree node expanded */
  int32_t sample;          /* 0 .. lambda-1 */
  float u[4];              /* sampled control */
  float x[12];             /* x' = PropagateODE(x, u, dt), the end of the segment (Alg. 2) */
  int32_t steps;           /* integration steps of the segment */
  int32_t fail_step;       /* first step whose state or swept box fails; steps + 1 if valid */
  int32_t valid;
  uint32_t cell;           /* sub-region of x' (region * 64 + index) */
  int32_t goal;            /* valid, accepted and in X_goal */
  int32_t accept;          /* added to V_U */
  int32_t new_id;          /* tree id given to the accepted sample, else -1 */
} kp_trace_record;

/* Bytes of workspace needed for `desc` (0 if desc is invalid). */
size_t kp_workspace_bytes(const kp_problem_desc* desc);

/* Bytes of trace buffer kp_expand needs for the current state. */
size_t kp_trace_bytes(const kp_problem* h);

/*
 * Alg. 1 set-up: checks the description, copies it and the obstacles,
 * carves the workspace and initialises the tree with the root x_init in V_E
 * and every P_accept = 1.  dev_workspace: device pointer, >= the size from
 * kp_workspace_bytes, borrowed for the handle's lifetime.  hip_stream: a
 * hipStream_t borrowed for the handle's lifetime.  Returns KP_E_START_INVALID
 * / KP_E_GOAL_INVALID when Problem 1's x_init in X_valid / X_goal in X_valid
 * fail.  On success *out receives the handle; synchronises the stream.
 */
kp_status kp_create_problem(const kp_problem_desc* desc, void* dev_workspace, size_t bytes,
                            void* hip_stream, kp_problem** out);

/* Frees the handle (not the workspace).  Synchronises the stream. */
kp_status kp_destroy_problem(kp_problem* h);

/* Back to Alg. 1 set-up with a new seed; the workspace is re-initialised. */
kp_status kp_reset(kp_problem* h, uint64_t seed);

/*
 * Alg. 2 (Propagate) with eq. (6): frontier V_E in ascending id order,
 * lambda, then |V_E| * lambda expansions (random control, PropagateODE,
 * validity, sub-region, n_valid / n_invalid, acceptance); accepted samples
 * are written after the tree's last node in (frontier position, sample)
 * order -- V_U, not yet part of T.  Enqueue only.  dev_trace: NULL or a
 * device buffer of kp_trace_bytes() bytes receiving one kp_trace_record per
 * lane.
 */
kp_status kp_expand(kp_problem* h, void* dev_trace);

/* Alg. 3 (UpdateEstimates, eqs. 3-5) over R_avail.  Enqueue only.
 * KP_E_ORDER unless called after kp_expand. */
kp_status kp_update_regions(kp_problem* h);

/*
 * Alg. 4 (UpdateNodeSets): V_E -> V_O with probability 1 - P_accept, V_U into
 * T and V_E with the goal test, V_O -> V_E with probability P_accept unless a
 * goal was found; then the next frontier and lambda.  goal_id: NULL (enqueue
 * only) or a host int receiving the goal node id or -1 (synchronises).
 * KP_E_ORDER unless called after kp_update_regions.
 */
kp_status kp_update_tree(kp_problem* h, int32_t* goal_id);

/* Alg. 1's loop until a goal node, a full tree, an empty frontier or the
 * time / iteration budget.  Synchronous. */
kp_status kp_plan(kp_problem* h, kp_plan_result* out);

/* Counters (synchronises the stream). */
kp_status kp_get_stats(kp_problem* h, kp_iter_stats* out);

/* Copy the whole state to host buffers (layout above).  Synchronous.
 * out->n_nodes and out->iteration are outputs; every array must hold
 * node_cap (node arrays) or R (region arrays) entries. */
kp_status kp_copy_tree(kp_problem* h, kp_tree_host* out);

/* Replace the state with a host copy (n_nodes >= 1, same layout); the next
 * call must be kp_expand.  Synchronous. */
kp_status kp_load_tree(kp_problem* h, const kp_tree_host* in);

/* Remark 1's adaptive t_e: move the tree of src (between iterations) into dst,
 * a handle of the same problem and seed with a capacity >= |T|, device to
 * device; dst then continues as if it had grown the tree itself (frontier
 * and eq. (6) recomputed with its capacity).  Synchronous. */
kp_status kp_transfer_tree(kp_problem* src, kp_problem* dst);

/* Node ids from the root to `node`: the parent walk behind the trajectory
 * that Alg. 4 returns when its goal test succeeds.  ids: host array of cap
 * entries; *len receives the path length.  KP_E_ARG if node is out of range
 * or the path exceeds cap. */
kp_status kp_get_path(kp_problem* h, int32_t node, int32_t* ids, int32_t cap, int32_t* len);

/* The trajectory from the root to `node` (Alg. 4 returns it for the goal
 * node): for each of the *len nodes of the path, row i of x holds its state
 * (n floats), row i of u the control of the edge into it (m floats, zero for
 * the root) and steps[i] that edge's integration steps (0 for the root; the
 * segment duration is steps[i] * h).  Host buffers of cap rows; any of x, u,
 * steps may be NULL (all NULL: only *len).  KP_E_ORDER in the middle of an
 * iteration; KP_E_ARG if node is out of range or the path exceeds cap.
 * Synchronous. */
kp_status kp_get_trajectory(kp_problem* h, int32_t node, float* x, float* u, int32_t* steps,
                            int32_t cap, int32_t* len);

/* Per-kernel timing with HIP events on the handle's stream (0 = off).  While
 * on, every launch carries two events stamped with its dispatch's begin and end; totals accumulate until
 * the next call with on = 1.  kp_kernel_times fills, for kernel index k
 * (0 propagate, 1 region estimates, 2 node sets, 3 frontier, 4 V_U commit, 5 the fused
 * commit + region + node-set pass that kp_plan runs after each propagate, 6 the learned
 * proposal's network over the frontier), the launch
 * count and the summed duration in milliseconds.  Synchronises. */
kp_status kp_set_profiling(kp_problem* h, int32_t on);
kp_status kp_kernel_times(kp_problem* h, int32_t kernel, int64_t* launches, double* total_ms);

/* Per-lane records of the expansions that kp_plan and kp_batch_plan run
 * (Alg. 2 inside Alg. 1's loop): with dev_trace set, every propagate launch
 * of the planning loop writes one kp_trace_record per lane of this problem,
 * as kp_expand does, overwriting the previous iteration's records (new_id
 * stays -1: ids are given in the fused pass after it).  dev_trace: NULL (off) or device memory of kp_trace_bytes()
 * bytes, 4-byte aligned, borrowed until replaced.  Used to compare the planning
 * loop lane by lane with a reference, one iteration per kp_plan call
 * (max_iters = 1). */
kp_status kp_set_trace(kp_problem* h, void* dev_trace);

/* Caps on the workgroups of every launch of the handle: prop_blocks for the
 * expansion, node_blocks for the V_U commit and the node passes (0 = the
 * occupancy maximum, the default).  Kernels take their work from ticket
 * counters or contiguous chunks and read their sizes from device memory, so
 * the results do not depend on these caps; small caps make one block serve
 * many tiles.  The node-set pass of kp_plan keeps at least one block per 16
 * node tiles (65,536 nodes) of the tree's bound, above the cap if need be. */
kp_status kp_set_launch_limits(kp_problem* h, int32_t prop_blocks, int32_t node_blocks);

const char* kp_status_str(kp_status s);
/* Text of the last error of handle h; with h = NULL, of the last failed call
 * on this thread that takes no handle and reports one (kp_mlp_train_noalloc). */
const char* kp_last_error(const kp_problem* h);

/* ---------------------------------------------------------------------------
 * Learned control proposal
 *
 * Alg. 2 draws every control uniformly from U.  With a proposal set on a
 * handle, expansion (iteration it, parent f, sample s) draws instead from a
 * Gaussian that a small network predicts for f, with probability mix, and
 * keeps the uniform draw otherwise.  The uniform share keeps a positive
 * density on all of U, which the completeness argument of Sec. V (Theorem 1)
 * relies on.
 *
 * Network: 16 inputs -> 128 -> 128 -> 8 outputs, relu after the two hidden
 * layers.  Parameters: one FP32 vector of KP_MLP_PARAMS floats, W1 [128][16],
 * b1 [128], W2 [128][128], b2 [128], W3 [8][128], b3 [8] (row-major, output
 * index first).  Every product takes BF16 operands (round to nearest even of
 * the FP32 weight or activation) and accumulates in FP32.
 *
 * Inputs of node x in region R: (raw_k - c_k) * s_k, raw = (x_0 .. x_{n-1},
 * P_accept(R) of eq. 5, goal_center - x_{0..2}, zeros).  c and s map the state
 * box to [-1, 1] and P_accept from [0, 1] to [-1, 1]; the goal offset is scaled
 * by 2 / (x_hi - x_lo) of the workspace; unused inputs are zero.
 *
 * Head, control j < m (c_j, r_j: centre and half-width of U):
 *   mean_j = c_j + r_j tanh(o_j),   std_j = r_j exp(clip(o_{4+j}, -4, 0)).
 * Draw: learned iff word 0 of Philox(it, f, s, 4) < floor(mix * 2^32); then
 * z_0, z_1 and z_2, z_3 are the Box-Muller transforms of words (0, 1) and
 * (2, 3) of Philox(it, f, s, 5), with u1 = ((a >> 8) + 1) 2^-24 and
 * u2 = (b >> 8) 2^-24; u_j = clip(mean_j + std_j z_j, u_lo_j, u_hi_j).
 *
 * Training objective: mean over a minibatch of
 *   sum_{j<m} [ (t_j - tanh o_j)^2 exp(-2 ls_j) / 2 + ls_j ],
 * ls_j = clip(o_{4+j}, -4, 0), t_j = (u_j - c_j) / r_j the logged control in
 * normalised units (the Gaussian negative log-likelihood up to constants).
 *
 * The functions without a handle return KP_E_ARG for bad arguments and
 * KP_E_DEVICE when a launch fails; they only enqueue on hip_stream.
 * ---------------------------------------------------------------------------*/
#define KP_MLP_INPUTS 16
#define KP_MLP_HIDDEN 128
#define KP_MLP_OUTPUTS 8
#define KP_MLP_PARAMS 19720
#define KP_MLP_PACKED_BYTES 87072   /* BF16 operand tiles + FP32 biases */
#define KP_MLP_BLOCK_ROWS 64        /* minibatch rows per partial gradient */

/* Convert FP32 parameters (device, KP_MLP_PARAMS floats) to the device layout
 * the kernels read (dev_packed: KP_MLP_PACKED_BYTES bytes, 16-byte aligned,
 * caller-owned).  Run again after every parameter change. */
kp_status kp_mlp_pack(const float* dev_params, void* dev_packed, void* hip_stream);

/* Raw outputs o (rows x 8 floats, device) of rows x 16 input features (device,
 * 16-byte aligned rows).  rows = 0 is a no-op. */
kp_status kp_mlp_forward(const void* dev_packed, const float* dev_x, int32_t rows, float* dev_out,
                         void* hip_stream);

/* Gradient of the training objective over one minibatch of `batch` rows
 * drawn from n_rows rows of features dev_x (n_rows x 16) and targets dev_t
 * (n_rows x 4; entries j >= n_ctrl ignored).  sample_key = 0: the minibatch is
 * rows 0 .. batch-1 (batch <= n_rows); otherwise row k of the minibatch is
 * (word 0 of Philox(step, k, 0, 6) with key sample_key) * n_rows >> 32.
 * Writes ceil(batch / KP_MLP_BLOCK_ROWS) partial gradients (KP_MLP_PARAMS
 * floats each, in parameter order; they sum to the gradient) to dev_partials
 * and as many partial losses (summing to the objective) to dev_loss. */
kp_status kp_mlp_grad(const void* dev_packed, const float* dev_x, const float* dev_t, int32_t n_rows,
                      int32_t n_ctrl, int32_t batch, uint64_t sample_key, int32_t step,
                      float* dev_partials, float* dev_loss, void* hip_stream);

/* Adam step `step` (1-based, bias-corrected; Kingma & Ba, 2015) on dev_params
 * with moments dev_m1, dev_m2 (KP_MLP_PARAMS floats each, zero before step 1),
 * the gradient being the sum of n_partials partial gradients (in order). */
kp_status kp_mlp_adam(float* dev_params, float* dev_m1, float* dev_m2, const float* dev_partials,
                      int32_t n_partials, int32_t step, float lr, float beta1, float beta2,
                      float eps, void* hip_stream);

/* `steps` rounds of kp_mlp_pack, kp_mlp_grad (random minibatches, steps
 * step0 .. step0+steps-1) and kp_mlp_adam (steps step0+1 ..).  dev_loss
 * receives steps x ceil(batch / KP_MLP_BLOCK_ROWS) partial losses; on return
 * dev_packed holds the updated parameters. */
kp_status kp_mlp_train(float* dev_params, float* dev_m1, float* dev_m2, void* dev_packed,
                       const float* dev_x, const float* dev_t, int32_t n_rows, int32_t n_ctrl,
                       int32_t batch, int32_t steps, int32_t step0, float lr, uint64_t sample_key,
                       float* dev_partials, float* dev_loss, void* hip_stream);

/* kp_mlp_train without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and results as
 * kp_mlp_train, minus dev_partials: the partial gradients of each step live
 * in a file-scope device array of the library that holds
 * KP_MLP_STATIC_MAX_BATCH / KP_MLP_BLOCK_ROWS partial gradients (32 x
 * KP_MLP_PARAMS floats, 2.5 MB).  Each GPU the library runs on holds its own
 * copy until the process ends; the first call on a GPU looks up its address
 * there (no allocation).  The call allocates nothing, on the device or the
 * host.
 *   batch > KP_MLP_STATIC_MAX_BATCH, or any argument kp_mlp_train refuses:
 *   KP_E_ARG, with the reason in kp_last_error(NULL) (per thread).
 * Every call on one GPU shares that GPU's array and it keeps the last call's
 * contents: calls that overlap on one GPU (two streams, two threads) race and
 * must not be made.  Each step writes every partial gradient it uses before
 * it reads it, so nothing needs to start at zero. */
#define KP_MLP_STATIC_MAX_BATCH 2048
kp_status kp_mlp_train_noalloc(float* dev_params, float* dev_m1, float* dev_m2, void* dev_packed,
                               const float* dev_x, const float* dev_t, int32_t n_rows,
                               int32_t n_ctrl, int32_t batch, int32_t steps, int32_t step0,
                               float lr, uint64_t sample_key, float* dev_loss, void* hip_stream);

/* Use the packed network dev_packed for the handle's expansions from the next
 * kp_expand / kp_plan on, mixed with the uniform draw at rate mix in [0, 1):
 * the uniform share 1 - mix must stay positive (KP_E_ARG otherwise), since it
 * is what keeps every control reachable (dev_packed = NULL or mix = 0:
 * uniform only).  dev_head: device scratch of
 * head_rows x 8 floats, head_rows >= node_cap.  Both buffers are borrowed
 * until the proposal is replaced.  KP_E_ORDER in the middle of an iteration.
 * Synchronises. */
kp_status kp_set_proposal(kp_problem* h, const void* dev_packed, float* dev_head, int64_t head_rows,
                          float mix);

/* Training rows from the tree path root -> node: row row0 + k holds the input
 * features of the parent of edge k (dev_x, 16 floats per row) and the edge's
 * control in normalised units (dev_t, 4 floats per row, zero past m), for
 * edges that fit below cap_rows.  *n_rows receives the rows written.
 * Synchronises. */
kp_status kp_log_path(kp_problem* h, int32_t node, float* dev_x, float* dev_t, int32_t cap_rows,
                      int32_t row0, int32_t* n_rows);

/* Training rows from every edge of the tree whose child lies strictly closer
 * to the goal centre than its parent (valid expansions that made progress),
 * in node id order: row row0 + k holds the parent's input features (dev_x)
 * and the edge's control in normalised units (dev_t), as kp_log_path writes
 * them, for rows below cap_rows.  *n_rows receives the rows written.  Must be
 * called between iterations (KP_E_ORDER otherwise).  Synchronises. */
kp_status kp_log_tree_edges(kp_problem* h, float* dev_x, float* dev_t, int32_t cap_rows,
                            int32_t row0, int32_t* n_rows);

/* ---------------------------------------------------------------------------
 * Batched planning
 *
 * Many independent problems advance together: every iteration kernel is
 * launched once for the whole batch, with one grid row per problem, and a
 * batch of iterations between two status reads can be replayed from a
 * captured HIP graph.  Each problem's work and result are exactly those of
 * kp_plan on that problem alone (the kernels' results do not depend on grid
 * shapes).  The problems must share dynamics and integrator; each must be
 * between iterations (after create, reset or kp_update_tree).
 * ---------------------------------------------------------------------------*/
typedef struct kp_batch kp_batch;

typedef struct {
  int32_t iters_per_sync;   /* iterations enqueued between status reads, 1..64 */
  int32_t use_graph;        /* 1: replay a captured HIP graph of those iterations */
  int32_t prop_blocks;      /* most propagate workgroups per problem and launch (>= 1) */
  int32_t node_blocks;      /* most commit / node-set workgroups per problem and launch (>= 1) */
} kp_batch_config;

/* Device workspace of a batch of n problems (the problem table and status). */
size_t kp_batch_workspace_bytes(int32_t n);

/* problems: n handles (borrowed for the batch's lifetime); dev_workspace:
 * device memory of kp_batch_workspace_bytes(n) bytes, 256-byte aligned,
 * borrowed.  The batch launches on a stream of its own (default priority)
 * after the work already queued on the first problem's stream.  The default
 * configuration uses the single-problem grid sizes and 8 iterations per read. */
kp_status kp_batch_create(kp_problem* const* problems, int32_t n, void* dev_workspace, size_t bytes,
                          kp_batch** out);
kp_status kp_batch_set_config(kp_batch* b, const kp_batch_config* cfg);
kp_status kp_batch_get_config(const kp_batch* b, kp_batch_config* cfg);

/* Alg. 1's loop for every problem of the batch until each one stops
 * (goal, full tree, empty frontier, or its own iteration / time budget).
 * results: n entries; elapsed_ms of entry i is the wall time from the call
 * until the status read that saw problem i stop.  *batch_ms (nullable): wall
 * time of the whole call.  Synchronous. */
kp_status kp_batch_plan(kp_batch* b, kp_plan_result* results, double* batch_ms);

/* SWITCHED OFF: every call returns KP_E_ARG (its first GPU run did not
 * finish and the cause is not yet known; see kp_batch_last_error).  Intended
 * behaviour: the same loop as kp_batch_plan in one persistent launch over a
 * device work queue (batched planning of Sec. IV-C's independent queries without a host
 * round trip per iteration).  Each workgroup takes the next problem from the
 * queue, largest node_cap first, and runs all of its iterations: expansion,
 * UpdateEstimates and UpdateNodeSets (Algs. 2-4), separated by workgroup
 * barriers, until the problem stops (goal, full tree, empty frontier, its
 * max_iters, or its t_max_ms measured on the device wall clock from the
 * moment a workgroup takes it).  Every problem's result and tree are exactly
 * those of kp_plan on it alone.  results: n entries; elapsed_ms of entry i is
 * the device time from the first workgroup's start to the end of problem i.
 * *batch_ms (nullable): wall time of the whole call.  Problems with a learned
 * proposal are refused (KP_E_ARG): use kp_batch_plan.  The batch
 * configuration (iterations per read, graphs, grid caps) does not apply.
 * Synchronous. */
kp_status kp_batch_plan_queue(kp_batch* b, kp_plan_result* results, double* batch_ms);

/* kp_reset of every problem of the batch (seeds: one per problem), enqueued
 * back to back with a single wait at the end. */
kp_status kp_batch_reset(kp_batch* b, const uint64_t* seeds);

kp_status kp_batch_destroy(kp_batch* b);
const char* kp_batch_last_error(const kp_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* KP_H */

// Internal definitions shared by the kernels (kp_kernels.hip) and the host
// library (kp_api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kp.h"

namespace kp {

// threads per propagate block: 16 waves, one block per compute unit at 4
// waves per SIMD.  Every block stages the obstacle table (and the grid) in
// its LDS, so fewer, larger blocks read that shared input fewer times.
__host__ __device__ constexpr int prop_block(int) { return 1024; }
// largest obstacle grid (u16 words: cell offsets and obstacle ids) a
// double-integrator block stages in LDS
constexpr int kGridMaxWords = 32768;
// double integrators with more obstacles than this use the grid; with fewer,
// a wave's candidate list is short or empty and costs less than a grid
// lookup at every step
constexpr int kGridMinObstacles = 64;
constexpr int kNodeBlock = 1024;     // threads per node-pass block
constexpr int kNodesPerThread = 4;   // nodes per thread in the node passes
constexpr int kNodeTile = kNodeBlock * kNodesPerThread;  // nodes per node-pass tile (4096)
constexpr int kChunkTiles = 256;     // 64-lane wave tiles per accepted-sample chunk sum
constexpr int kChunkTilesMax = 16;   // node tiles a k_post block takes as one chunk (4 V_E bits each in a u64)
constexpr int kRegionBlock = 1024;   // threads of the single region-estimate block
constexpr int kRegionsPerBlock = 4 * 1024;  // regions per region block of k_post (4 per thread of 1024)
// region blocks at the start of a k_post grid row
__host__ __device__ constexpr int post_region_blocks(int R) {
  return (R + kRegionsPerBlock - 1) / kRegionsPerBlock;
}
constexpr int kCommitBlock = 1024;   // threads per commit block (16 waves)
constexpr int kMaxPath = 65536;      // longest path kp_get_path can return
constexpr int kDoneNone = 0;
constexpr int32_t kNoGoal = 0x7fffffff;

// Device control block: sizes and counters of the running iteration.  Written
// only by single threads (finalisers) or by atomics, read at block start.
// Counters that many blocks update sit in kGroups separate 128-byte lines
// (group = block index mod kGroups): same-address atomics from the whole
// chip serialise, about 11 ns each, so one shared line would throttle them.
constexpr int kGroups = 8;
struct alignas(128) TotLine {
  // lanes, valid lanes, integration steps, swept-box tests, and the steps
  // whose state and swept box were tested (a lane stops testing at its first
  // failing step but integrates on to the end of its segment)
  unsigned long long lanes, valid, steps, box, checked;
};
struct alignas(128) TkLine {
  uint32_t v;
};
struct alignas(256) Ctl {
  int32_t N;          // |T|
  int32_t nF;         // |V_E| for the next expansion
  int32_t lambda;     // eq. (6)
  int32_t lanes;      // nF * lambda
  int32_t nU;         // |V_U| of the last expansion
  int32_t it;         // iteration number (Philox counter word 0)
  int32_t goal_id;    // smallest new node id in X_goal, kNoGoal if none
  int32_t done;       // 0 running, else KP_SOLVED / KP_TREE_FULL / KP_FRONTIER_EMPTY
  uint32_t epoch;     // tags look-back status words; bumped once per iteration
  uint32_t tk_front, tk_nodes;   // tile tickets of the node passes
  uint32_t bd_front, bd_nodes;   // blocks finished (last-block finalisation)
  uint32_t err;       // nonzero: a device check failed (a wait hit its spin limit, a grid too small)
  uint32_t iters_done;
  // the iteration as k_commit saw it, read by k_nodesets (whose finaliser
  // rewrites N, it, epoch and done while other blocks may still start)
  int32_t sN, snU, sit, sdone;
  uint32_t sepoch;
  // frontier list: entries e < f_expl are F[e]; entries e >= f_expl are the
  // ids f_base + (e - f_expl) (the last admission, kept implicit by k_post)
  int32_t f_expl, f_base;
  uint32_t region_ready;  // epoch whose thresholds k_post's region block has written
  uint32_t goal_hit;      // an accepted sample of this query reached X_goal
  // the iteration as k_propagate found it, read by k_post (whose finaliser
  // rewrites the fields above while other blocks may still start)
  int32_t slanes, slam;
  // region pass of k_post over several blocks: the largest score (bits of a
  // non-negative double), the sum of the scaled scores, and the blocks that
  // have added to each and written their thresholds; k_propagate clears them
  alignas(128) unsigned long long rg_max;
  unsigned long long rg_sum;
  uint32_t rg_cnt_max, rg_cnt_sum, rg_cnt_thr;
  TotLine tot[kGroups];  // propagate totals per group; the host adds the groups
  TkLine tkp[kGroups];   // propagate tile tickets per group; cleared by k_commit / k_post
};
static_assert(sizeof(Ctl) <= 4096, "control block size");

// Problem constants, passed by value to every kernel.
struct Params {
  int32_t n, m, K, cap;
  int32_t lambda_max, n_obs, S, R;
  int32_t dur_mode;         // 1: segment of 1 + (w * K >> 32) steps, w = word 1 of tag 1
  int32_t box_sym;          // quadcopter state box symmetric about zero outside position
  int32_t G[3];
  int32_t na[3];        // fine cells per axis = G * S
  float h, margin, goal_r2, rc;
  // quadcopter: a segment's displacement from accelerations, per axis, lies
  // in [ra_lo, ra_hi] (a_lo (K h)^2 / 2 .. a_hi (K h)^2 / 2 around 0)
  float ra_lo[3], ra_hi[3];
  float goal_c[3];
  float w_lo[3];        // workspace lower corner
  float inv_w[3];       // fine cells per unit length
  alignas(64) float x_lo[12];   // 64-byte aligned: one wide scalar load each
  alignas(64) float x_hi[12];
  float u_lo[4], u_hi[4];
  float mass, grav, Ixx, Iyy, Izz;
  float inv_m, inv_Ixx, inv_Iyy, inv_Izz;
  float dIyz, dIzx, dIxy;   // Iyy - Izz, Izz - Ixx, Ixx - Iyy
  uint32_t key0, key1;
  // obstacle grid of the double integrator (og_n[0] = 0: none): og_n cells
  // per axis of width 1 / og_inv from og_org; og_words u16 words
  int32_t og_n[3];
  int32_t og_words;
  float og_org[3];
  float og_inv;
  double delta, eps;
  // learned proposal: a sample takes the network's Gaussian when its mixture
  // word is below mix_thr (0: uniform only); network inputs are
  // (raw feature - fc) * fs
  unsigned long long mix_thr;
  float fc[16], fs[16];
};

struct TraceRec {
  int32_t parent, sample;
  float u[4];
  float x[12];
  int32_t steps, fail_step, valid;
  uint32_t cell;
  int32_t goal, accept, new_id;
};
static_assert(sizeof(TraceRec) == 100, "trace record layout");

// Device pointers carved from the caller's workspace.
struct Dev {
  Ctl* ctl;
  float* x;            // [n][capP]
  float* u;            // [m][capP]
  int32_t* parent;     // [capP]
  uint32_t* cell;      // [capP]
  uint8_t* flag;       // [capP]  1 = V_E
  int32_t* birth;      // [capP]
  uint8_t* sample;     // [capP]
  int32_t* F;          // [capP] frontier list
  unsigned long long* nv;       // [R]
  unsigned long long* ni;       // [R]
  unsigned long long* visited;  // [R]
  unsigned long long* thr;      // [R]
  uint8_t* avail;      // [R]
  float* obs;          // [6][n_obs] SoA
  // obstacle grid (double integrator): u16 offsets of the cells' lists
  // [ncell + 1], then the lists' obstacle ids; padded to an even count
  const uint16_t* og;
  unsigned long long* st_front;  // look-back status, one word per tile
  unsigned long long* st_nodes;
  // accepted samples staged per 64-lane wave tile: slot = tile * 64 + rank
  float* sx;           // [n][capP]
  float* su;           // [m][capP]
  uint32_t* scell;     // [capP]
  uint32_t* slane;     // [capP] lane index << 1 | goal bit
  int32_t* spar;       // [capP] parent id (the commit never reads F, which the
                       // node-set pass of the same launch rewrites)
  uint32_t* scount;    // [node_cap / 64 + 2] accepted samples per 64-lane wave tile
  uint32_t* ssum;      // [2][nchunk] accepted samples per kChunkTiles consecutive wave
                       // tiles; iteration it uses half it & 1
  int32_t* path;       // [kMaxPath + 1]
  const uint4* mlp;    // packed network (kp_mlp_pack layout), borrowed; null if uniform
  float* head;         // [rows][8] Gaussian mean (4) and std (4) per frontier entry, borrowed
  TraceRec* trace;     // per-lane records of the planning loop's expansions (kp_set_trace), or null
  int32_t capP;        // padded node capacity (multiple of kNodeTile)
  int32_t tiles_node;  // entries of st_front / st_nodes
  int32_t nchunk;      // entries of ssum
  int32_t pad;
};


// Everything a kernel needs besides per-launch arguments; lives in device
// memory (start of the workspace) so kernels read it through one pointer
// with scalar loads instead of holding a large by-value argument in registers.
struct Env {
  Params p;
  Dev d;
};

// Launchers (kp_kernels.hip).  Each returns the hipError_t of the launch.
// A non-null Timing pair is filled with the dispatch's own begin and end
// timestamps (hipExtLaunchKernel), so that the measured span is the kernel
// alone, without the command-processor work between two event markers.
struct Vec12 { float v[12]; };
struct Timing {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
hipError_t launch_zero(const Params& p, const Dev& d, const Env* env, hipStream_t s);
hipError_t launch_root(const Env* env, Vec12 x_init, hipStream_t s);
hipError_t launch_frontier(const Env* env, int grid, hipStream_t s, Timing t);
hipError_t launch_propagate(int dyn, int integ, int sym, const Env* env, size_t lds,
                            TraceRec* trace, int grid, hipStream_t s, Timing t);
hipError_t launch_commit(const Env* env, TraceRec* trace, int grid, int with_region,
                         hipStream_t s, Timing t);
hipError_t launch_region(const Env* env, hipStream_t s, Timing t);
// n_region: post_region_blocks(R) (the largest over a batch)
hipError_t launch_post(const Env* env, int n_region, int n_commit, int n_nodes, hipStream_t s,
                       Timing t);
hipError_t launch_nodesets(const Env* env, int grid, hipStream_t s, Timing t);
hipError_t launch_path(const Env* env, int32_t node, hipStream_t s);
// rows of kTrajWords words (state, control, steps) of the path k_path wrote
constexpr int kTrajRowWords = 17;
hipError_t launch_path_gather(const Env* env, int32_t len, float* out, hipStream_t s);

// batched planning: one grid row (blockIdx.y) per problem of an Env* table
struct BatchStatus {
  int32_t done, N, nF, lanes, iters_done, goal_id, err, pad;
  unsigned long long lanes_total, valid_total;
};
hipError_t launch_propagate_batch(int dyn, int integ, int sym, const Env* const* envs, int n,
                                  size_t lds, int grid, hipStream_t s);
hipError_t launch_post_batch(const Env* const* envs, int n, int n_region, int n_commit,
                             int n_nodes, hipStream_t s);
hipError_t launch_batch_status(const Env* const* envs, int n, BatchStatus* out, hipStream_t s);

// batched planning in one launch over a device work queue (k_plan_queue):
// per problem its iteration budget and its time budget in wall-clock ticks
// (0: none); the queue head and the earliest block start; then, written by
// the kernel, each problem's end tick and iterations run
constexpr int kQueueBlock = 1024;
struct QueueJob {
  int32_t iters;
  int32_t pad;
  unsigned long long ticks;
};
struct QueueCtl {
  uint32_t head;
  uint32_t pad;
  unsigned long long t_start;
};
hipError_t launch_plan_queue(int dyn, int integ, int sym, const Env* const* envs,
                             const int32_t* order, const QueueJob* jobs, int n, QueueCtl* qc,
                             unsigned long long* t_end, int32_t* ran, size_t lds, int grid,
                             hipStream_t s);
// dynamic LDS of one problem in k_plan_queue (propagate body at kQueueBlock threads)
size_t queue_lds_bytes(int dyn, int n_obs, int grid_words);
int occupancy_queue(int dyn, int integ, int sym, size_t lds, int* blocks_per_cu);
hipError_t launch_set_done(const Env* env, int32_t code, hipStream_t s);
hipError_t launch_set_ctl(const Env* env, int32_t N, int32_t it, hipStream_t s);

// learned proposal (kp_mlp.hip)
constexpr int kMlpIn = 16, kMlpHid = 128, kMlpOut = 8;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid +
                           kMlpOut * kMlpHid + kMlpOut;
constexpr int kMlpRowsPerBlock = 64;  // rows per training block (one partial gradient each)
size_t mlp_packed_bytes();
hipError_t launch_mlp_pack(const float* params, uint4* packed, hipStream_t s);
hipError_t launch_mlp_forward(const uint4* packed, const float* x, int32_t rows, float* out,
                              hipStream_t s);
hipError_t launch_mlp_head(const Env* env, int grid, hipStream_t s, Timing t);
hipError_t launch_mlp_head_batch(const Env* const* envs, int n, int grid, hipStream_t s);
int mlp_head_grid_max(int cu_count);
int mlp_head_rows_per_block();
hipError_t launch_mlp_grad(const uint4* packed, const float* x, const float* t, int32_t n_rows,
                           int32_t m, int32_t batch, uint64_t key, int32_t step, float* partials,
                           float* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* params, float* m1, float* m2, const float* partials,
                           int32_t n_partials, float lr, float beta1, float beta2, float eps,
                           float inv_bc1, float inv_bc2, hipStream_t s);
hipError_t launch_log_path(const Env* env, float* x, float* t, int32_t cap_rows, int32_t row0,
                           hipStream_t s);
int edge_tiles(int32_t n_nodes);
hipError_t launch_edge_count(const Env* env, int tiles, uint32_t* tcount, hipStream_t s);
hipError_t launch_edge_write(const Env* env, int tiles, const uint32_t* tcount, float* x, float* t,
                             int32_t cap_rows, int32_t row0, hipStream_t s);
int occupancy_propagate(int dyn, int integ, int sym, size_t lds, int* blocks_per_cu);
int occupancy_nodes(int* blocks_per_cu);
int occupancy_commit(int* blocks_per_cu);
int occupancy_post(int* blocks_per_cu);
size_t propagate_lds_bytes(int dyn, int n_obs, int grid_words);

}  // namespace kp

// Host side of the C ABI declared in include/kp.h: argument checks, workspace
// carving, the Alg. 1 loop, state copies and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kp.h"
#include "kp_internal.h"

using namespace kp;

namespace {
// Text of the last failed call without a handle, per thread (kp_last_error(NULL)).
thread_local char g_call_err[256] = "";

void call_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_call_err, sizeof g_call_err, fmt, ap);
  va_end(ap);
}

constexpr size_t kAlign = 256;
constexpr int kProfKernels = 7;  // propagate, region, node sets, frontier, commit, fused post,
                                  // proposal network
constexpr int kEventPool = 512;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  size_t ctl, env, x, u, parent, cell, flag, birth, sample, F;
  size_t nv, ni, visited, thr, avail, obs, st_front, st_nodes, path;
  size_t sx, su, scell, slane, spar, scount, ssum, og;
  size_t total;
  int capP, tiles_node, nchunk;
};

int state_dim(int dyn) { return dyn == KP_DYN_DI6 ? 6 : 12; }
int ctrl_dim(int dyn) { return dyn == KP_DYN_DI6 ? 3 : 4; }

// Returns an empty string if the description is acceptable.
std::string check_desc(const kp_problem_desc* d) {
  if (!d) return "desc is NULL";
  if (d->abi_version != KP_ABI_VERSION) return "abi_version mismatch";
  if (d->dynamics != KP_DYN_DI6 && d->dynamics != KP_DYN_QUAD12) return "unknown dynamics";
  if (d->integrator != KP_INT_EULER && d->integrator != KP_INT_RK4) return "unknown integrator";
  if (d->steps < 1 || d->steps > 4096) return "steps must be in [1, 4096]";
  if (!(d->h > 0.0f) || !std::isfinite(d->h)) return "h must be positive";
  if (d->n_obstacles < 0 || d->n_obstacles > KP_MAX_OBSTACLES) return "n_obstacles out of range";
  if (d->n_obstacles > 0 && !d->obstacles) return "obstacles is NULL";
  if (!(d->margin >= 0.0f)) return "margin must be >= 0";
  for (int a = 0; a < 3; ++a) {
    if (d->grid[a] < 1) return "grid entries must be >= 1";
    if (!(d->x_hi[a] > d->x_lo[a])) return "workspace bounds must satisfy x_lo < x_hi";
  }
  if ((long long)d->grid[0] * d->grid[1] * d->grid[2] > 65536) return "more than 65536 regions";
  if ((long long)d->grid[0] * d->sub > 1 << 20 || (long long)d->grid[1] * d->sub > 1 << 20 ||
      (long long)d->grid[2] * d->sub > 1 << 20)
    return "too many cells per axis";
  if (d->sub < 1 || d->sub > 4) return "sub must be in [1, 4]";
  if (d->node_cap < 1 || d->node_cap > (1 << 30)) return "node_cap must be in [1, 2^30]";
  if (d->lambda_max < 1 || d->lambda_max > 255) return "lambda_max must be in [1, 255]";
  if (!(d->delta > 0.0)) return "delta must be > 0";
  if (!(d->epsilon > 0.0) || d->epsilon > 1.0) return "epsilon must be in (0, 1]";
  const int n = state_dim(d->dynamics), m = ctrl_dim(d->dynamics);
  for (int j = 0; j < m; ++j)
    if (!(d->u_hi[j] >= d->u_lo[j])) return "control box must satisfy u_lo <= u_hi";
  for (int i = 0; i < n; ++i)
    if (!(d->x_hi[i] >= d->x_lo[i])) return "state box must satisfy x_lo <= x_hi";
  if (!(d->goal_radius >= 0.0f)) return "goal_radius must be >= 0";
  if (d->max_iters < 0) return "max_iters must be >= 0";
  if (d->iters_per_sync < 0 || d->iters_per_sync > 4096) return "iters_per_sync out of range";
  if (d->duration_mode != 0 && d->duration_mode != 1) return "duration_mode must be 0 or 1";
  if (d->reserved != 0) return "reserved must be 0";
  return std::string();
}

// Uniform grid over the workspace that lists, per cell, the obstacles a
// swept box touching the cell may hit (a double integrator among more than
// kGridMinObstacles boxes; other problems cull per tile instead).  Cells are cubes of width 1 / inv from org
// (the workspace grown by the margin and a little more), the index of
// coordinate x on axis a is floor((x - org_a) * inv) clamped to the grid,
// and an obstacle is listed in every cell of the index range of its own box,
// each end widened by 1e-3 of a cell.  The kernel widens the index range of a
// swept box the same way; a point that a swept box shares with an obstacle
// then lies in a cell that the kernel visits and that lists the obstacle, as
// long as the kernel's FP32 index map errs by less than 1e-3 of a cell (it
// errs by a few units in the last place).  The grid is the finest of a few
// sizes whose words (cell offsets, then ids, u16) fit kGridMaxWords, with at
// most max(64, 16 n_obs) cells.
struct ObsGrid {
  int n[3] = {0, 0, 0};
  float org[3] = {0.0f, 0.0f, 0.0f};
  float inv = 0.0f;
  std::vector<uint16_t> words;  // offsets [ncell + 1], then obstacle ids; even length
};

ObsGrid build_obs_grid(const kp_problem_desc* d) {
  ObsGrid g;
  if (d->dynamics != KP_DYN_DI6 || d->n_obstacles <= kGridMinObstacles) return g;
  const int no = d->n_obstacles;
  double lo[3], ext = 0.0, span[3];
  for (int a = 0; a < 3; ++a) {
    const double big = std::fmax(std::fabs((double)d->x_lo[a]), std::fabs((double)d->x_hi[a]));
    const double pad = (double)d->margin + 1e-3 * (1.0 + big);
    lo[a] = (double)d->x_lo[a] - pad;
    span[a] = ((double)d->x_hi[a] + pad) - lo[a];
    ext = std::fmax(ext, span[a]);
  }
  static const int kCells[] = {32, 24, 20, 16, 12, 10, 8, 6, 5, 4, 3, 2, 1};
  for (const int gm : kCells) {
    const float inv = (float)((double)gm / ext);
    const double invd = (double)inv;
    int n[3];
    float org[3];
    long long ncell = 1;
    for (int a = 0; a < 3; ++a) {
      org[a] = (float)lo[a];
      n[a] = (int)std::ceil(((double)lo[a] + span[a] - (double)org[a]) * invd);
      if (n[a] < 1) n[a] = 1;
      ncell *= n[a];
    }
    if (gm > 1 && (ncell > std::max<long long>(64, 16LL * no) || ncell + 1 > kGridMaxWords))
      continue;
    // cell index range of each obstacle, per axis
    std::vector<int> rng((size_t)6 * (no > 0 ? no : 1));
    for (int k = 0; k < no; ++k) {
      for (int a = 0; a < 3; ++a) {
        auto idx = [&](double x, double slack) {
          const double t = std::floor((x - (double)org[a]) * invd + slack);
          return (int)std::fmin(std::fmax(t, 0.0), (double)(n[a] - 1));
        };
        const double olo = d->obstacles[6 * k + a], ohi = d->obstacles[6 * k + 3 + a];
        const int i0 = idx(std::fmin(olo, ohi), -1e-3), i1 = idx(std::fmax(olo, ohi), 1e-3);
        rng[6 * k + a] = i0;
        rng[6 * k + 3 + a] = i1;
      }
    }
    std::vector<uint32_t> cnt((size_t)ncell + 1, 0u);
    long long total = 0;
    for (int k = 0; k < no; ++k) {
      const int* r = &rng[6 * k];
      for (int z = r[2]; z <= r[5]; ++z)
        for (int y = r[1]; y <= r[4]; ++y)
          for (int x = r[0]; x <= r[3]; ++x) ++cnt[((size_t)z * n[1] + y) * n[0] + x];
      total += (long long)(r[3] - r[0] + 1) * (r[4] - r[1] + 1) * (r[5] - r[2] + 1);
    }
    if (gm > 1 && ncell + 1 + total > kGridMaxWords) continue;
    g.words.assign((size_t)(ncell + 1 + total + 1) & ~(size_t)1, 0);
    uint32_t off = 0;
    for (long long c = 0; c < ncell; ++c) {
      g.words[(size_t)c] = (uint16_t)off;
      off += cnt[(size_t)c];
    }
    g.words[(size_t)ncell] = (uint16_t)off;
    std::vector<uint32_t> fill(g.words.begin(), g.words.begin() + ncell);
    uint16_t* ids = g.words.data() + ncell + 1;
    for (int k = 0; k < no; ++k) {  // ascending ids in every list
      const int* r = &rng[6 * k];
      for (int z = r[2]; z <= r[5]; ++z)
        for (int y = r[1]; y <= r[4]; ++y)
          for (int x = r[0]; x <= r[3]; ++x) ids[fill[((size_t)z * n[1] + y) * n[0] + x]++] = (uint16_t)k;
    }
    for (int a = 0; a < 3; ++a) {
      g.n[a] = n[a];
      g.org[a] = org[a];
    }
    g.inv = inv;
    return g;
  }
  return g;  // not reached: one cell always fits
}

Layout make_layout(const kp_problem_desc* d) {
  Layout L{};
  const int n = state_dim(d->dynamics), m = ctrl_dim(d->dynamics);
  const size_t R = (size_t)d->grid[0] * d->grid[1] * d->grid[2];
  const size_t capP = align_up((size_t)d->node_cap + 1, kNodeTile);
  L.capP = (int)capP;
  L.tiles_node = (int)(capP / kNodeTile + 2);
  L.nchunk = (int)(((size_t)d->node_cap / 64 + 2 + kChunkTiles - 1) / kChunkTiles);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, kAlign);
    return o;
  };
  L.ctl = take(sizeof(Ctl));
  L.env = take(sizeof(Env));
  L.x = take(capP * n * 4);
  L.u = take(capP * m * 4);
  L.parent = take(capP * 4);
  L.cell = take(capP * 4);
  L.flag = take(capP);
  L.birth = take(capP * 4);
  L.sample = take(capP);
  L.F = take(capP * 4);
  L.nv = take(R * 8);
  L.ni = take(R * 8);
  L.visited = take(R * 8);
  L.thr = take(R * 8);
  L.avail = take(R);
  L.obs = take((size_t)(d->n_obstacles > 0 ? d->n_obstacles : 1) * 6 * 4);
  L.st_front = take((size_t)L.tiles_node * 8);
  L.st_nodes = take((size_t)L.tiles_node * 8);
  L.path = take((size_t)(kMaxPath + 1) * 4);
  L.sx = take(capP * n * 4);
  L.su = take(capP * m * 4);
  L.scell = take(capP * 4);
  L.slane = take(capP * 4);
  L.spar = take(capP * 4);
  L.scount = take(((size_t)d->node_cap / 64 + 2) * 4);  // one count per 64-lane wave tile
  L.ssum = take((size_t)L.nchunk * 2 * 4);
  L.og = take(build_obs_grid(d).words.size() * 2 + 4);
  L.total = off;
  return L;
}

// Distance-squared from a point to a closed box, in double.
double point_box_d2(const double* c, const double* lo, const double* hi) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double t = 0.0;
    if (c[a] < lo[a]) t = lo[a] - c[a];
    else if (c[a] > hi[a]) t = c[a] - hi[a];
    d2 += t * t;
  }
  return d2;
}

}  // namespace

struct kp_problem {
  kp_problem_desc desc;
  std::vector<float> obs;  // row-major copy
  ObsGrid og;              // double integrator: obstacle grid (uploaded at create)
  size_t lds_prop = 0;     // dynamic LDS of a propagate block
  Params prm;
  Dev dev;
  Env* env_dev;  // device copy of {prm, dev} read by the kernels
  Env env_host;
  Layout L;
  hipStream_t stream;
  int n, m, R;
  int cu_count;
  int grid_prop_max;
  int grid_node_max;
  int grid_post_max;   // k_post blocks resident at once (its node-set blocks are capped by it)
  int grid_commit_max;
  int grid_head_max;
  int lim_prop = 0, lim_node = 0;  // kp_set_launch_limits caps (0: none)
  TraceRec* plan_trace = nullptr;  // kp_set_trace: per-lane records of kp_plan's expansions
  int stage;  // 0: next is kp_expand; 1: next is kp_update_regions; 2: next is kp_update_tree
  bool ctl_fresh = false;  // hctl holds the device control block (no launch since the last read)
  Ctl* hctl;  // pinned host mirror of the control block
  std::string err;
  // profiling
  bool prof;
  hipEvent_t ev[kEventPool][2];
  int ev_kernel[kEventPool];
  int ev_used;
  long long prof_launches[kProfKernels];
  double prof_ms[kProfKernels];
  bool events_made;
};

namespace {

// the fields of two descriptions that shape a tree (all but capacity, budgets
// and the obstacle pointer), compared one by one
bool same_problem(const kp_problem_desc& a, const kp_problem_desc& b) {
  auto eq = [](const void* x, const void* y, size_t n) { return std::memcmp(x, y, n) == 0; };
  return a.dynamics == b.dynamics && a.integrator == b.integrator && a.steps == b.steps &&
         eq(&a.h, &b.h, sizeof a.h) && eq(a.dyn_params, b.dyn_params, sizeof a.dyn_params) &&
         eq(a.u_lo, b.u_lo, sizeof a.u_lo) && eq(a.u_hi, b.u_hi, sizeof a.u_hi) &&
         eq(a.x_lo, b.x_lo, sizeof a.x_lo) && eq(a.x_hi, b.x_hi, sizeof a.x_hi) &&
         a.n_obstacles == b.n_obstacles && eq(&a.margin, &b.margin, sizeof a.margin) &&
         eq(a.x_init, b.x_init, sizeof a.x_init) &&
         eq(a.goal_center, b.goal_center, sizeof a.goal_center) &&
         eq(&a.goal_radius, &b.goal_radius, sizeof a.goal_radius) &&
         eq(a.grid, b.grid, sizeof a.grid) && a.sub == b.sub && a.lambda_max == b.lambda_max &&
         eq(&a.delta, &b.delta, sizeof a.delta) && eq(&a.epsilon, &b.epsilon, sizeof a.epsilon) &&
         a.seed == b.seed && a.duration_mode == b.duration_mode;
}

kp_status fail(kp_problem* h, kp_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

kp_status hip_fail(kp_problem* h, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, KP_E_DEVICE, msg);
}

// True when the quadcopter's state box is symmetric about zero in every
// coordinate but position (lo = -hi exactly): the kernel then tests those
// coordinates as |x| <= hi, one compare instead of two.
bool quad_box_symmetric(const kp_problem_desc& d) {
  if (d.dynamics != KP_DYN_QUAD12) return false;
  for (int i = 3; i < 12; ++i)
    if (!(d.x_lo[i] == -d.x_hi[i])) return false;
  return true;
}

void fill_params(kp_problem* h) {
  const kp_problem_desc& d = h->desc;
  Params& p = h->prm;
  std::memset(&p, 0, sizeof(p));
  p.n = h->n;
  p.m = h->m;
  p.K = d.steps;
  p.cap = d.node_cap;
  p.lambda_max = d.lambda_max;
  p.n_obs = d.n_obstacles;
  p.S = d.sub;
  p.R = h->R;
  for (int a = 0; a < 3; ++a) {
    p.G[a] = d.grid[a];
    p.na[a] = d.grid[a] * d.sub;
    p.w_lo[a] = d.x_lo[a];
    p.inv_w[a] = (float)((double)p.na[a] / ((double)d.x_hi[a] - (double)d.x_lo[a]));
    p.goal_c[a] = d.goal_center[a];
  }
  p.h = d.h;
  p.margin = d.margin;
  p.goal_r2 = d.goal_radius * d.goal_radius;
  for (int i = 0; i < 12; ++i) {
    p.x_lo[i] = d.x_lo[i];
    p.x_hi[i] = d.x_hi[i];
  }
  for (int j = 0; j < 4; ++j) {
    p.u_lo[j] = d.u_lo[j];
    p.u_hi[j] = d.u_hi[j];
  }
  p.mass = d.dyn_params[0];
  p.grav = d.dyn_params[1];
  p.Ixx = d.dyn_params[2];
  p.Iyy = d.dyn_params[3];
  p.Izz = d.dyn_params[4];
  p.inv_m = 1.0f / p.mass;
  p.inv_Ixx = 1.0f / p.Ixx;
  p.inv_Iyy = 1.0f / p.Iyy;
  p.inv_Izz = 1.0f / p.Izz;
  p.dIyz = p.Iyy - p.Izz;
  p.dIzx = p.Izz - p.Ixx;
  p.dIxy = p.Ixx - p.Iyy;
  p.dur_mode = d.duration_mode;
  p.box_sym = quad_box_symmetric(d) ? 1 : 0;
  p.key0 = (uint32_t)d.seed;
  p.key1 = (uint32_t)(d.seed >> 32);
  for (int a = 0; a < 3; ++a) {
    p.og_n[a] = h->og.n[a];
    p.og_org[a] = h->og.org[a];
  }
  p.og_inv = h->og.inv;
  p.og_words = (int32_t)h->og.words.size();
  p.delta = d.delta;
  p.eps = d.epsilon;
  // Culling radius: a step is collision-checked only when it starts from a
  // state inside the velocity bounds, so each step moves a position by at
  // most h * (v_max + h * a_max) per axis (Euler: h * v_max).
  const int vo = (d.dynamics == KP_DYN_DI6) ? 3 : 6;
  double vmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    vmax = std::fmax(vmax, std::fabs((double)d.x_lo[vo + a]));
    vmax = std::fmax(vmax, std::fabs((double)d.x_hi[vo + a]));
  }
  double amax = 0.0;
  if (d.dynamics == KP_DYN_DI6) {
    for (int j = 0; j < 3; ++j)
      amax = std::fmax(amax, std::fmax(std::fabs((double)d.u_lo[j]), std::fabs((double)d.u_hi[j])));
  } else {
    const double tmax = std::fmax(std::fabs((double)d.u_lo[0]), std::fabs((double)d.u_hi[0]));
    amax = tmax / std::fabs((double)d.dyn_params[0]) + std::fabs((double)d.dyn_params[1]);
  }
  // learned proposal off; input affine map of the network's features
  p.mix_thr = 0ull;
  for (int k = 0; k < 16; ++k) {
    p.fc[k] = 0.0f;
    p.fs[k] = 0.0f;
  }
  for (int k = 0; k < h->n; ++k) {
    p.fc[k] = (float)(0.5 * ((double)d.x_lo[k] + (double)d.x_hi[k]));
    p.fs[k] = (d.x_hi[k] > d.x_lo[k]) ? (float)(2.0 / ((double)d.x_hi[k] - (double)d.x_lo[k])) : 0.0f;
  }
  p.fc[h->n] = 0.5f;
  p.fs[h->n] = 2.0f;
  for (int a = 0; a < 3; ++a)
    p.fs[h->n + 1 + a] = (float)(2.0 / ((double)d.x_hi[a] - (double)d.x_lo[a]));
  const double hh = d.h;
  const double per_step = (d.integrator == KP_INT_EULER) ? hh * vmax : hh * (vmax + hh * amax);
  double rc = d.steps * per_step * (1.0 + 1e-4) + 1e-3;
  if (!std::isfinite(rc)) rc = 3.0e38;
  p.rc = (float)rc;
  // Quadcopter: how far accelerations move a position over a whole segment,
  // away from the straight line of the start velocity.  The acceleration is
  // thrust / m times a column of a rotation matrix (entries in [-1, 1]) less
  // g along z, so per axis it lies in [-A, A] (x, y) and [-A - g, A - g] (z),
  // A = max |thrust| / m; j steps add at most a (j h)^2 / 2 of either sign.
  if (d.dynamics == KP_DYN_QUAD12) {
    const double tk = d.steps * hh;
    const double A = std::fmax(std::fabs((double)d.u_lo[0]), std::fabs((double)d.u_hi[0])) /
                     std::fabs((double)d.dyn_params[0]);
    const double g = d.dyn_params[1];
    for (int a = 0; a < 3; ++a) {
      const double alo = -A - (a == 2 ? g : 0.0), ahi = A - (a == 2 ? g : 0.0);
      double lo = std::fmin(alo, 0.0) * 0.5 * tk * tk * (1.0 + 1e-4) - 1e-4;
      double hi = std::fmax(ahi, 0.0) * 0.5 * tk * tk * (1.0 + 1e-4) + 1e-4;
      if (!std::isfinite(lo)) lo = -3.0e38;
      if (!std::isfinite(hi)) hi = 3.0e38;
      p.ra_lo[a] = (float)lo;
      p.ra_hi[a] = (float)hi;
    }
  }
}

void carve(kp_problem* h, void* ws) {
  char* b = static_cast<char*>(ws);
  const Layout& L = h->L;
  Dev& v = h->dev;
  v.ctl = reinterpret_cast<Ctl*>(b + L.ctl);
  h->env_dev = reinterpret_cast<Env*>(b + L.env);
  v.x = reinterpret_cast<float*>(b + L.x);
  v.u = reinterpret_cast<float*>(b + L.u);
  v.parent = reinterpret_cast<int32_t*>(b + L.parent);
  v.cell = reinterpret_cast<uint32_t*>(b + L.cell);
  v.flag = reinterpret_cast<uint8_t*>(b + L.flag);
  v.birth = reinterpret_cast<int32_t*>(b + L.birth);
  v.sample = reinterpret_cast<uint8_t*>(b + L.sample);
  v.F = reinterpret_cast<int32_t*>(b + L.F);
  v.nv = reinterpret_cast<unsigned long long*>(b + L.nv);
  v.ni = reinterpret_cast<unsigned long long*>(b + L.ni);
  v.visited = reinterpret_cast<unsigned long long*>(b + L.visited);
  v.thr = reinterpret_cast<unsigned long long*>(b + L.thr);
  v.avail = reinterpret_cast<uint8_t*>(b + L.avail);
  v.obs = reinterpret_cast<float*>(b + L.obs);
  v.og = reinterpret_cast<const uint16_t*>(b + L.og);
  v.st_front = reinterpret_cast<unsigned long long*>(b + L.st_front);
  v.st_nodes = reinterpret_cast<unsigned long long*>(b + L.st_nodes);
  v.path = reinterpret_cast<int32_t*>(b + L.path);
  v.mlp = nullptr;
  v.head = nullptr;
  v.sx = reinterpret_cast<float*>(b + L.sx);
  v.su = reinterpret_cast<float*>(b + L.su);
  v.scell = reinterpret_cast<uint32_t*>(b + L.scell);
  v.slane = reinterpret_cast<uint32_t*>(b + L.slane);
  v.spar = reinterpret_cast<int32_t*>(b + L.spar);
  v.scount = reinterpret_cast<uint32_t*>(b + L.scount);
  v.ssum = reinterpret_cast<uint32_t*>(b + L.ssum);
  v.capP = L.capP;
  v.tiles_node = L.tiles_node;
  v.nchunk = L.nchunk;
}

kp_status sync_ctl(kp_problem* h) {
  hipError_t e = hipMemcpyAsync(h->hctl, h->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "status copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
  if (const uint32_t err = h->hctl->err) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "device check failed (bits 0x%x: 1 frontier look-back wait limit, 2 commit id "
                  "past |T| + lanes, 4 node-set look-back wait limit, 8 estimates wait limit, 16 "
                  "node-set grid below one block per chunk)",
                  err);
    return fail(h, KP_E_DEVICE, msg);
  }
  h->ctl_fresh = true;
  return KP_OK;
}

// propagate totals, kept per counter group on the device
struct Totals {
  unsigned long long lanes = 0, valid = 0, steps = 0, box = 0, checked = 0;
};
Totals totals(const Ctl& c) {
  Totals t;
  for (int g = 0; g < kGroups; ++g) {
    t.lanes += c.tot[g].lanes;
    t.valid += c.tot[g].valid;
    t.steps += c.tot[g].steps;
    t.box += c.tot[g].box;
    t.checked += c.tot[g].checked;
  }
  return t;
}

// profiling: hand a launch a pair of events that the runtime stamps with the
// dispatch's begin and end
Timing prof_slot(kp_problem* h, int kernel) {
  Timing t;
  if (!h->prof || h->ev_used >= kEventPool) return t;
  const int k = h->ev_used++;
  h->ev_kernel[k] = kernel;
  t.start = h->ev[k][0];
  t.stop = h->ev[k][1];
  return t;
}
void prof_collect(kp_problem* h) {
  if (!h->prof || h->ev_used == 0) return;
  (void)hipStreamSynchronize(h->stream);
  for (int k = 0; k < h->ev_used; ++k) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->ev[k][0], h->ev[k][1]) == hipSuccess) {
      h->prof_ms[h->ev_kernel[k]] += ms;
      h->prof_launches[h->ev_kernel[k]] += 1;
    }
  }
  h->ev_used = 0;
}

// workgroup caps of a launch: the occupancy maxima, lowered by
// kp_set_launch_limits (results do not depend on them)
int cap_prop(const kp_problem* h) {
  return (h->lim_prop > 0 && h->lim_prop < h->grid_prop_max) ? h->lim_prop : h->grid_prop_max;
}
int cap_node(const kp_problem* h) {
  return (h->lim_node > 0 && h->lim_node < h->grid_node_max) ? h->lim_node : h->grid_node_max;
}
// a propagate grid of g blocks rounded up to a multiple of 8 when g >= 8,
// not above gmax rounded down to one
int xcd_grid(int g, int gmax) {
  if (g < 8) return g;
  const int up = (g + 7) & ~7, cap = gmax & ~7;
  return up <= cap ? up : (cap >= 8 ? cap : g);
}
int cap_post_nodes(const kp_problem* h) {
  return (h->lim_node > 0 && h->lim_node < h->grid_post_max) ? h->lim_node : h->grid_post_max;
}
int cap_commit(const kp_problem* h) {
  return (h->lim_node > 0 && h->lim_node < h->grid_commit_max) ? h->lim_node : h->grid_commit_max;
}

// n_nodes: |T| as the host knows it (exact: reset or a loaded tree)
kp_status do_frontier(kp_problem* h, long long n_nodes) {
  h->ctl_fresh = false;
  const long long tiles = (n_nodes + kNodeTile - 1) / kNodeTile;
  const int gmax = cap_node(h);
  int grid = (int)(tiles < gmax ? tiles : gmax);
  if (grid < 1) grid = 1;
  hipError_t e = launch_frontier(h->env_dev, grid, h->stream, prof_slot(h, 3));
  if (e != hipSuccess) return hip_fail(h, e, "frontier launch");
  return KP_OK;
}

// grids from the last host-known sizes (exact after a status read; upper
// bounds otherwise -- the kernels read the true sizes from device memory)
// with_region: the commit launch also runs Alg. 3 in one extra block (kp_plan)
// with_commit false: the caller follows with do_post (kp_plan)
kp_status do_propagate(kp_problem* h, TraceRec* trace, long long lanes_ub, bool with_commit) {
  h->ctl_fresh = false;
  // one block per 64-lane tile up to the cap (the kernel hands the first
  // tiles to wave 0 of every block), a multiple of 8 blocks from 8 on (the
  // kernel gives each XCD a contiguous range of them)
  long long tiles = (lanes_ub + 63) / 64;
  const int gmax = cap_prop(h);
  int grid = (int)(tiles < gmax ? tiles : gmax);
  if (grid < 1) grid = 1;
  grid = xcd_grid(grid, gmax);
  hipError_t e = launch_propagate(h->desc.dynamics, h->desc.integrator, h->prm.box_sym, h->env_dev,
                                  h->lds_prop, trace, grid, h->stream, prof_slot(h, 0));
  if (e != hipSuccess) return hip_fail(h, e, "propagate launch");
  if (!with_commit) return KP_OK;
  const long long ctiles = (lanes_ub + kCommitBlock - 1) / kCommitBlock;
  const int cmax = cap_commit(h);
  int cgrid = (int)(ctiles < cmax ? ctiles : cmax);
  if (cgrid < 1) cgrid = 1;
  e = launch_commit(h->env_dev, trace, cgrid, 0, h->stream, prof_slot(h, 4));
  if (e != hipSuccess) return hip_fail(h, e, "commit launch");
  return KP_OK;
}

// k_post after a propagate launch: commit, region and node-set blocks sized
// from the host's bounds on the expansion and on the old tree
kp_status do_post(kp_problem* h, long long lanes_ub, long long old_nodes_ub) {
  h->ctl_fresh = false;
  const long long ctiles = (lanes_ub + kCommitBlock - 1) / kCommitBlock;
  const long long ntiles = (old_nodes_ub + kNodeTile - 1) / kNodeTile;
  // commit blocks take at most half of the resident k_post blocks, so a wide
  // expansion leaves room for the node-set blocks that follow them in the grid
  const int chalf = h->grid_post_max / 2 > 0 ? h->grid_post_max / 2 : 1;
  const int cmax = cap_commit(h) < chalf ? cap_commit(h) : chalf, nmax = cap_post_nodes(h);
  const int nc = (int)(ctiles < cmax ? ctiles : cmax);
  // node-set blocks: up to the cap, but at least one per kChunkTilesMax tiles
  int nn = (int)(ntiles < nmax ? ntiles : nmax);
  if (ntiles > (long long)kChunkTilesMax * nn) nn = (int)((ntiles + kChunkTilesMax - 1) / kChunkTilesMax);
  hipError_t e = launch_post(h->env_dev, post_region_blocks(h->R), nc, nn, h->stream,
                             prof_slot(h, 5));
  if (e != hipSuccess) return hip_fail(h, e, "post launch");
  return KP_OK;
}

// the proposal network over the frontier (before a propagate launch), when a
// learned proposal is set; nf_ub bounds |V_E|
kp_status do_head(kp_problem* h, long long nf_ub) {
  if (h->prm.mix_thr == 0ull) return KP_OK;
  h->ctl_fresh = false;
  const long long rpb = mlp_head_rows_per_block();
  const long long blocks = (nf_ub + rpb - 1) / rpb;
  int grid = (int)(blocks < h->grid_head_max ? blocks : h->grid_head_max);
  if (grid < 1) grid = 1;
  hipError_t e = launch_mlp_head(h->env_dev, grid, h->stream, prof_slot(h, 6));
  if (e != hipSuccess) return hip_fail(h, e, "proposal launch");
  return KP_OK;
}

kp_status do_region(kp_problem* h) {
  h->ctl_fresh = false;
  hipError_t e = launch_region(h->env_dev, h->stream, prof_slot(h, 1));
  if (e != hipSuccess) return hip_fail(h, e, "region launch");
  return KP_OK;
}

kp_status do_nodesets(kp_problem* h, long long nodes_ub) {
  h->ctl_fresh = false;
  long long tiles = (nodes_ub + kNodeTile - 1) / kNodeTile;
  const int gmax = cap_node(h);
  int grid = (int)(tiles < gmax ? tiles : gmax);
  if (grid < 1) grid = 1;
  hipError_t e = launch_nodesets(h->env_dev, grid, h->stream, prof_slot(h, 2));
  if (e != hipSuccess) return hip_fail(h, e, "node sets launch");
  return KP_OK;
}

// copy {prm, dev} to the device (stream-ordered; the host copy lives in the
// handle, and callers synchronise before returning)
hipError_t upload_env(kp_problem* h) {
  h->env_host.p = h->prm;
  h->env_host.d = h->dev;
  return hipMemcpyAsync(h->env_dev, &h->env_host, sizeof(Env), hipMemcpyHostToDevice, h->stream);
}

kp_status init_state(kp_problem* h) {
  h->ctl_fresh = false;
  hipError_t e = upload_env(h);
  if (e != hipSuccess) return hip_fail(h, e, "environment upload");
  e = launch_zero(h->prm, h->dev, h->env_dev, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "zero launch");
  Vec12 xi;
  for (int k = 0; k < 12; ++k) xi.v[k] = h->desc.x_init[k];
  e = launch_root(h->env_dev, xi, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "root launch");
  kp_status st = do_frontier(h, 1);
  if (st != KP_OK) return st;
  h->stage = 0;
  return sync_ctl(h);
}

}  // namespace

extern "C" {

size_t kp_workspace_bytes(const kp_problem_desc* desc) {
  if (!check_desc(desc).empty()) return 0;
  return make_layout(desc).total;
}

size_t kp_trace_bytes(const kp_problem* h) {
  if (!h) return 0;
  return (size_t)h->desc.node_cap * sizeof(TraceRec);
}

kp_status kp_create_problem(const kp_problem_desc* desc, void* dev_workspace, size_t bytes,
                            void* hip_stream, kp_problem** out) {
  if (!out) return KP_E_ARG;
  *out = nullptr;
  const std::string why = check_desc(desc);
  if (!why.empty()) return KP_E_ARG;
  if (!dev_workspace) return KP_E_ARG;
  const Layout L = make_layout(desc);
  if (bytes < L.total || (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) != 0)
    return KP_E_WORKSPACE;
  // Problem 1 requires x_init in X_valid and X_goal inside X_valid.
  const int n = state_dim(desc->dynamics);
  for (int i = 0; i < n; ++i) {
    const float v = desc->x_init[i];
    if (!std::isfinite(v) || v < desc->x_lo[i] || v > desc->x_hi[i]) return KP_E_START_INVALID;
  }
  double xi[3] = {desc->x_init[0], desc->x_init[1], desc->x_init[2]};
  double gc[3] = {desc->goal_center[0], desc->goal_center[1], desc->goal_center[2]};
  const double mg = desc->margin;
  for (int k = 0; k < desc->n_obstacles; ++k) {
    const float* o = desc->obstacles + 6 * k;
    double lo[3] = {o[0] - mg, o[1] - mg, o[2] - mg};
    double hi[3] = {o[3] + mg, o[4] + mg, o[5] + mg};
    if (point_box_d2(xi, lo, hi) == 0.0) return KP_E_START_INVALID;
  }
  for (int a = 0; a < 3; ++a) {
    if (gc[a] - desc->goal_radius < desc->x_lo[a] || gc[a] + desc->goal_radius > desc->x_hi[a])
      return KP_E_GOAL_INVALID;
  }
  for (int k = 0; k < desc->n_obstacles; ++k) {
    const float* o = desc->obstacles + 6 * k;
    double lo[3] = {o[0], o[1], o[2]};
    double hi[3] = {o[3], o[4], o[5]};
    const double r = (double)desc->goal_radius + mg;
    if (point_box_d2(gc, lo, hi) <= r * r) return KP_E_GOAL_INVALID;
  }

  kp_problem* h = new (std::nothrow) kp_problem();
  if (!h) return KP_E_ARG;
  h->desc = *desc;
  h->desc.obstacles = nullptr;
  h->obs.assign(desc->obstacles, desc->obstacles + (size_t)6 * desc->n_obstacles);
  h->og = build_obs_grid(desc);
  h->lds_prop = propagate_lds_bytes(desc->dynamics, desc->n_obstacles, (int)h->og.words.size());
  h->n = n;
  h->m = ctrl_dim(desc->dynamics);
  h->R = desc->grid[0] * desc->grid[1] * desc->grid[2];
  h->L = L;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->prof = false;
  h->ev_used = 0;
  h->events_made = false;
  for (int k = 0; k < kProfKernels; ++k) {
    h->prof_launches[k] = 0;
    h->prof_ms[k] = 0.0;
  }
  fill_params(h);
  carve(h, dev_workspace);

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete h;
    return KP_E_DEVICE;
  }
  int bp = 1, bn = 1, bc = 1, bpo = 1;
  occupancy_propagate(desc->dynamics, desc->integrator, h->prm.box_sym, h->lds_prop, &bp);
  occupancy_nodes(&bn);
  occupancy_commit(&bc);
  occupancy_post(&bpo);
  h->grid_prop_max = bp * h->cu_count;
  h->grid_node_max = bn * h->cu_count;
  h->grid_post_max = bpo * h->cu_count;
  h->grid_commit_max = bc * h->cu_count;
  h->grid_head_max = mlp_head_grid_max(h->cu_count);
  if (hipHostMalloc(reinterpret_cast<void**>(&h->hctl), sizeof(Ctl), hipHostMallocDefault) !=
      hipSuccess) {
    delete h;
    return KP_E_DEVICE;
  }
  std::memset(h->hctl, 0, sizeof(Ctl));
  // obstacles as SoA: lo x[], lo y[], lo z[], hi x[], hi y[], hi z[]
  std::vector<float> soa((size_t)6 * (desc->n_obstacles > 0 ? desc->n_obstacles : 1), 0.0f);
  for (int k = 0; k < desc->n_obstacles; ++k)
    for (int c = 0; c < 6; ++c) soa[(size_t)c * desc->n_obstacles + k] = h->obs[(size_t)6 * k + c];
  e = hipMemcpyAsync(h->dev.obs, soa.data(), soa.size() * sizeof(float), hipMemcpyHostToDevice,
                     h->stream);
  if (e == hipSuccess && !h->og.words.empty())
    e = hipMemcpyAsync(const_cast<uint16_t*>(h->dev.og), h->og.words.data(),
                       h->og.words.size() * sizeof(uint16_t), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->dev.ctl, 0, sizeof(Ctl), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipHostFree(h->hctl);
    delete h;
    return KP_E_DEVICE;
  }
  kp_status st = init_state(h);
  if (st != KP_OK) {
    (void)hipHostFree(h->hctl);
    delete h;
    return st;
  }
  *out = h;
  return KP_OK;
}

kp_status kp_destroy_problem(kp_problem* h) {
  if (!h) return KP_E_ARG;
  (void)hipStreamSynchronize(h->stream);
  if (h->events_made) {
    for (int k = 0; k < kEventPool; ++k) {
      (void)hipEventDestroy(h->ev[k][0]);
      (void)hipEventDestroy(h->ev[k][1]);
    }
  }
  (void)hipHostFree(h->hctl);
  delete h;
  return KP_OK;
}

kp_status kp_reset(kp_problem* h, uint64_t seed) {
  if (!h) return KP_E_ARG;
  h->desc.seed = seed;
  h->prm.key0 = (uint32_t)seed;
  h->prm.key1 = (uint32_t)(seed >> 32);
  return init_state(h);
}

kp_status kp_expand(kp_problem* h, void* dev_trace) {
  if (!h) return KP_E_ARG;
  if (h->stage != 0) return fail(h, KP_E_ORDER, "kp_expand must follow kp_update_tree");
  const long long ub = (long long)h->desc.node_cap - h->hctl->N;
  kp_status st = do_head(h, h->desc.node_cap);
  if (st != KP_OK) return st;
  st = do_propagate(h, static_cast<TraceRec*>(dev_trace), ub > 0 ? ub : 1, true);
  if (st != KP_OK) return st;
  h->stage = 1;
  return KP_OK;
}

kp_status kp_update_regions(kp_problem* h) {
  if (!h) return KP_E_ARG;
  if (h->stage != 1) return fail(h, KP_E_ORDER, "kp_update_regions must follow kp_expand");
  kp_status st = do_region(h);
  if (st != KP_OK) return st;
  h->stage = 2;
  return KP_OK;
}

kp_status kp_update_tree(kp_problem* h, int32_t* goal_id) {
  if (!h) return KP_E_ARG;
  if (h->stage != 2) return fail(h, KP_E_ORDER, "kp_update_tree must follow kp_update_regions");
  kp_status st = do_nodesets(h, h->desc.node_cap);
  if (st != KP_OK) return st;
  h->stage = 0;
  if (goal_id) {
    st = sync_ctl(h);
    if (st != KP_OK) return st;
    *goal_id = (h->hctl->goal_id == kNoGoal) ? -1 : h->hctl->goal_id;
  }
  return KP_OK;
}

kp_status kp_plan(kp_problem* h, kp_plan_result* out) {
  if (!h || !out) return KP_E_ARG;
  if (h->stage != 0) return fail(h, KP_E_ORDER, "kp_plan must start after a complete iteration");
  std::memset(out, 0, sizeof(*out));
  const auto t0 = std::chrono::steady_clock::now();
  kp_status st = h->ctl_fresh ? KP_OK : sync_ctl(h);  // the mirror is current after a reset
  if (st != KP_OK) return st;
  const uint32_t it0 = h->hctl->iters_done;
  // Default: 8 iterations between status reads.  Every kernel reads its
  // sizes from the device and an oversized grid costs no atomics, so the
  // host round trip (about 13 us) is paid once per 8 iterations instead of
  // once per iteration; after a stop the rest of a batch is empty launches.
  const int per_sync = h->desc.iters_per_sync > 0 ? h->desc.iters_per_sync : 8;
  const long long cap = h->desc.node_cap;
  int status = KP_TIMEOUT;
  for (;;) {
    const Ctl& c = *h->hctl;
    if (c.done) {
      status = c.done;
      break;
    }
    const long long done_iters = (long long)c.iters_done - it0;
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (done_iters >= h->desc.max_iters || ms >= h->desc.t_max_ms) break;
    long long batch = per_sync;
    if (batch > h->desc.max_iters - done_iters) batch = h->desc.max_iters - done_iters;
    for (long long b = 0; b < batch; ++b) {
      // exact sizes for the first iteration of a batch, bounds after it
      const long long lanes_ub = (b == 0) ? c.lanes : cap - c.N;
      const long long old_nodes_ub = (b == 0) ? (long long)c.N : cap;
      if ((st = do_head(h, (b == 0) ? (long long)c.nF : cap)) != KP_OK) return st;
      if ((st = do_propagate(h, h->plan_trace, lanes_ub, false)) != KP_OK) return st;
      if ((st = do_post(h, lanes_ub, old_nodes_ub)) != KP_OK) return st;
    }
    if ((st = sync_ctl(h)) != KP_OK) return st;
    prof_collect(h);
  }
  const Ctl& c = *h->hctl;
  out->elapsed_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  out->status = status;
  out->goal_id = (c.goal_id == kNoGoal) ? -1 : c.goal_id;
  out->iterations = (int32_t)(c.iters_done - it0);
  out->n_nodes = c.N;
  const Totals t = totals(c);
  out->lanes_total = t.lanes;
  out->valid_total = t.valid;
  out->path_len = 0;
  if (out->goal_id >= 0) {
    int32_t len = 0;
    if (kp_get_path(h, out->goal_id, nullptr, 0, &len) == KP_OK) out->path_len = len;
  }
  return (kp_status)status;
}

kp_status kp_get_stats(kp_problem* h, kp_iter_stats* out) {
  if (!h || !out) return KP_E_ARG;
  hipError_t e = hipMemcpyAsync(h->hctl, h->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stats copy");
  const Ctl& c = *h->hctl;
  out->n_nodes = c.N;
  out->n_frontier = c.nF;
  out->lambda = c.lambda;
  out->iteration = c.it;
  out->goal_id = (c.goal_id == kNoGoal) ? -1 : c.goal_id;
  out->done_code = c.done;
  out->n_new = c.nU;
  out->device_error = (int32_t)c.err;
  const Totals t = totals(c);
  out->lanes_total = t.lanes;
  out->valid_total = t.valid;
  out->invalid_total = t.lanes - t.valid;
  out->steps_total = t.steps;
  out->box_tests_total = t.box;
  out->checked_steps_total = t.checked;
  out->grid_propagate = h->grid_prop_max;
  out->grid_nodes = h->grid_node_max;
  return KP_OK;
}

kp_status kp_copy_tree(kp_problem* h, kp_tree_host* o) {
  if (!h || !o || !o->x || !o->u || !o->parent || !o->cell || !o->flag || !o->birth ||
      !o->sample || !o->nv || !o->ni || !o->visited || !o->avail || !o->thr)
    return fail(h, KP_E_ARG, "kp_copy_tree: null buffer");
  kp_status st = sync_ctl(h);
  if (st != KP_OK) return st;
  // after kp_expand the accepted samples (V_U) already sit after the tree
  const int32_t N = h->hctl->N + (h->stage == 0 ? 0 : h->hctl->nU);
  o->n_nodes = N;
  o->iteration = h->hctl->it;
  const size_t pitch = (size_t)h->L.capP * 4;
  hipError_t e = hipSuccess;
  if (N > 0) {
    e = hipMemcpy2DAsync(o->x, (size_t)N * 4, h->dev.x, pitch, (size_t)N * 4, h->n,
                         hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(o->u, (size_t)N * 4, h->dev.u, pitch, (size_t)N * 4, h->m,
                           hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(o->parent, h->dev.parent, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(o->cell, h->dev.cell, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(o->flag, h->dev.flag, (size_t)N, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(o->birth, h->dev.birth, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(o->sample, h->dev.sample, (size_t)N, hipMemcpyDeviceToHost, h->stream);
  }
  const size_t R = (size_t)h->R;
  if (e == hipSuccess) e = hipMemcpyAsync(o->nv, h->dev.nv, R * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(o->ni, h->dev.ni, R * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o->visited, h->dev.visited, R * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(o->avail, h->dev.avail, R, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(o->thr, h->dev.thr, R * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "tree copy");
  return KP_OK;
}

kp_status kp_load_tree(kp_problem* h, const kp_tree_host* in) {
  if (!h || !in || !in->x || !in->u || !in->parent || !in->cell || !in->flag || !in->birth ||
      !in->sample || !in->nv || !in->ni || !in->visited || !in->avail || !in->thr)
    return fail(h, KP_E_ARG, "kp_load_tree: null buffer");
  const int32_t N = in->n_nodes;
  if (N < 1 || N > h->desc.node_cap || in->iteration < 0)
    return fail(h, KP_E_ARG, "kp_load_tree: n_nodes out of range");
  for (int32_t i = 0; i < N; ++i) {
    if (in->parent[i] >= i || (i > 0 && in->parent[i] < 0) || (i == 0 && in->parent[0] != -1))
      return fail(h, KP_E_ARG, "kp_load_tree: parent links must point to smaller ids");
    if ((in->cell[i] >> 6) >= (uint32_t)h->R)
      return fail(h, KP_E_ARG, "kp_load_tree: cell out of range");
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  const size_t pitch = (size_t)h->L.capP * 4;
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(h->dev.x, pitch, in->x, (size_t)N * 4, (size_t)N * 4, h->n,
                         hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(h->dev.u, pitch, in->u, (size_t)N * 4, (size_t)N * 4, h->m,
                         hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev.parent, in->parent, (size_t)N * 4, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev.cell, in->cell, (size_t)N * 4, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev.flag, in->flag, (size_t)N, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev.birth, in->birth, (size_t)N * 4, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev.sample, in->sample, (size_t)N, hipMemcpyHostToDevice, h->stream);
  const size_t R = (size_t)h->R;
  if (e == hipSuccess) e = hipMemcpyAsync(h->dev.nv, in->nv, R * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->dev.ni, in->ni, R * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev.visited, in->visited, R * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->dev.avail, in->avail, R, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->dev.thr, in->thr, R * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "tree load");
  h->ctl_fresh = false;
  e = launch_set_ctl(h->env_dev, N, in->iteration, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "control load");
  kp_status st = do_frontier(h, N);
  if (st != KP_OK) return st;
  h->stage = 0;
  return sync_ctl(h);
}

kp_status kp_transfer_tree(kp_problem* src, kp_problem* dst) {
  if (!src || !dst || src == dst) return KP_E_ARG;
  // every field that shapes the tree must agree; capacity and budgets may differ
  if (!same_problem(src->desc, dst->desc) || src->obs != dst->obs)
    return fail(dst, KP_E_ARG, "kp_transfer_tree: problems differ beyond their capacity");
  if (src->stage != 0) return fail(dst, KP_E_ORDER, "kp_transfer_tree: source mid-iteration");
  kp_status st = sync_ctl(src);
  if (st != KP_OK) return fail(dst, st, src->err);
  const int32_t N = src->hctl->N;
  const int32_t it = src->hctl->it;
  if (N > dst->desc.node_cap)
    return fail(dst, KP_E_ARG, "kp_transfer_tree: tree larger than the capacity");
  hipError_t e = hipStreamSynchronize(dst->stream);
  // device to device on the destination's stream; the source is idle (synchronised above)
  const size_t ps = (size_t)src->L.capP * 4, pd = (size_t)dst->L.capP * 4;
  hipStream_t s = dst->stream;
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(dst->dev.x, pd, src->dev.x, ps, (size_t)N * 4, dst->n,
                         hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(dst->dev.u, pd, src->dev.u, ps, (size_t)N * 4, dst->m,
                         hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.parent, src->dev.parent, (size_t)N * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.cell, src->dev.cell, (size_t)N * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.flag, src->dev.flag, (size_t)N, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.birth, src->dev.birth, (size_t)N * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.sample, src->dev.sample, (size_t)N, hipMemcpyDeviceToDevice, s);
  const size_t R = (size_t)dst->R;
  if (e == hipSuccess) e = hipMemcpyAsync(dst->dev.nv, src->dev.nv, R * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dst->dev.ni, src->dev.ni, R * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.visited, src->dev.visited, R * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->dev.avail, src->dev.avail, R, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dst->dev.thr, src->dev.thr, R * 8, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(dst, e, "tree transfer");
  dst->ctl_fresh = false;
  e = launch_set_ctl(dst->env_dev, N, it, s);
  if (e != hipSuccess) return hip_fail(dst, e, "control load");
  st = do_frontier(dst, N);
  if (st != KP_OK) return st;
  dst->stage = 0;
  return sync_ctl(dst);
}

kp_status kp_get_path(kp_problem* h, int32_t node, int32_t* ids, int32_t cap, int32_t* len) {
  if (!h || !len) return KP_E_ARG;
  kp_status st = sync_ctl(h);
  if (st != KP_OK) return st;
  if (node < 0 || node >= h->hctl->N) return fail(h, KP_E_ARG, "kp_get_path: node out of range");
  hipError_t e = launch_path(h->env_dev, node, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "path launch");
  int32_t n = 0;
  e = hipMemcpyAsync(&n, h->dev.path, 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "path length copy");
  *len = n;
  if (n > kMaxPath) return fail(h, KP_E_ARG, "kp_get_path: path longer than the path buffer");
  if (!ids) return KP_OK;
  if (n > cap) return fail(h, KP_E_ARG, "kp_get_path: ids buffer too small");
  e = hipMemcpyAsync(ids, h->dev.path + 1, (size_t)n * 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "path copy");
  return KP_OK;
}

kp_status kp_get_trajectory(kp_problem* h, int32_t node, float* x, float* u, int32_t* steps,
                            int32_t cap, int32_t* len) {
  if (!h || !len) return KP_E_ARG;
  if (h->stage != 0) return fail(h, KP_E_ORDER, "kp_get_trajectory in the middle of an iteration");
  int32_t n = 0;
  kp_status st = kp_get_path(h, node, nullptr, 0, &n);
  if (st != KP_OK) return st;
  *len = n;
  if (!x && !u && !steps) return KP_OK;
  if (n > cap) return fail(h, KP_E_ARG, "kp_get_trajectory: buffers too small");
  // the rows are gathered into the V_U staging area, unused between iterations
  if ((size_t)n * kTrajRowWords > (size_t)h->dev.capP * (size_t)h->n)
    return fail(h, KP_E_ARG, "kp_get_trajectory: path longer than the staging area holds");
  hipError_t e = launch_path_gather(h->env_dev, n, h->dev.sx, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "path gather launch");
  std::vector<float> rows((size_t)n * kTrajRowWords);
  e = hipMemcpyAsync(rows.data(), h->dev.sx, rows.size() * sizeof(float), hipMemcpyDeviceToHost,
                     h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "trajectory copy");
  for (int32_t i = 0; i < n; ++i) {
    const float* r = rows.data() + (size_t)i * kTrajRowWords;
    if (x)
      for (int k = 0; k < h->n; ++k) x[(size_t)i * h->n + k] = r[k];
    if (u)
      for (int j = 0; j < h->m; ++j) u[(size_t)i * h->m + j] = r[12 + j];
    if (steps) std::memcpy(&steps[i], &r[16], 4);
  }
  return KP_OK;
}

kp_status kp_set_profiling(kp_problem* h, int32_t on) {
  if (!h) return KP_E_ARG;
  prof_collect(h);
  if (on && !h->events_made) {
    for (int k = 0; k < kEventPool; ++k) {
      if (hipEventCreate(&h->ev[k][0]) != hipSuccess || hipEventCreate(&h->ev[k][1]) != hipSuccess)
        return fail(h, KP_E_DEVICE, "event creation failed");
    }
    h->events_made = true;
  }
  if (on) {
    for (int k = 0; k < kProfKernels; ++k) {
      h->prof_launches[k] = 0;
      h->prof_ms[k] = 0.0;
    }
  }
  h->prof = on != 0;
  return KP_OK;
}

kp_status kp_set_trace(kp_problem* h, void* dev_trace) {
  if (!h) return KP_E_ARG;
  if (dev_trace && (reinterpret_cast<uintptr_t>(dev_trace) & 3u))
    return fail(h, KP_E_ARG, "kp_set_trace: buffer not 4-byte aligned");
  h->plan_trace = static_cast<TraceRec*>(dev_trace);
  h->dev.trace = h->plan_trace;  // batched launches read it from the device environment
  hipError_t e = upload_env(h);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "environment upload");
  return KP_OK;
}

kp_status kp_set_launch_limits(kp_problem* h, int32_t prop_blocks, int32_t node_blocks) {
  if (!h) return KP_E_ARG;
  if (prop_blocks < 0 || node_blocks < 0)
    return fail(h, KP_E_ARG, "kp_set_launch_limits: negative workgroup count");
  h->lim_prop = prop_blocks;
  h->lim_node = node_blocks;
  return KP_OK;
}

kp_status kp_kernel_times(kp_problem* h, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!h || !launches || !total_ms || kernel < 0 || kernel >= kProfKernels) return KP_E_ARG;
  prof_collect(h);
  *launches = h->prof_launches[kernel];
  *total_ms = h->prof_ms[kernel];
  return KP_OK;
}

const char* kp_status_str(kp_status s) {
  switch (s) {
    case KP_OK: return "ok";
    case KP_SOLVED: return "solved";
    case KP_TIMEOUT: return "timeout";
    case KP_TREE_FULL: return "tree full";
    case KP_FRONTIER_EMPTY: return "frontier empty";
    case KP_E_ARG: return "invalid argument";
    case KP_E_DEVICE: return "device error";
    case KP_E_WORKSPACE: return "workspace too small or misaligned";
    case KP_E_START_INVALID: return "x_init is not a valid state";
    case KP_E_GOAL_INVALID: return "goal region is not inside the valid set";
    case KP_E_ORDER: return "call out of order";
  }
  return "unknown status";
}

const char* kp_last_error(const kp_problem* h) { return h ? h->err.c_str() : g_call_err; }

// ---------------------------------------------------------------------------
// learned proposal
// ---------------------------------------------------------------------------
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // extern "C"

// Partial gradients of kp_mlp_train_noalloc: a file-scope device array, one
// copy per GPU, in place of a caller workspace.  Host code never passes the
// array's name to a kernel (on the host it only stands in for the symbol);
// it passes the device address that hipGetSymbolAddress gives on each GPU.
namespace {
constexpr int kStaticPartials = KP_MLP_STATIC_MAX_BATCH / KP_MLP_BLOCK_ROWS;
static_assert(KP_MLP_STATIC_MAX_BATCH % KP_MLP_BLOCK_ROWS == 0, "whole partial blocks");
constexpr int kMaxDevices = 64;
std::mutex g_partials_mu;
float* g_partials_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) float scratch[(size_t)kStaticPartials * KP_MLP_PARAMS];

namespace {
// The device address of `scratch` on the GPU that stream s runs on, looked
// up once per GPU with that GPU current.
kp_status static_partials(hipStream_t s, float** out) {
  int dev = -1;
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    call_error("kp_mlp_train_noalloc: no device for the stream (%s)", hipGetErrorString(e));
    return KP_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_partials_mu);
  if (!g_partials_ptr[dev]) {
    int cur = -1;
    e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess || !ptr) {
      call_error("kp_mlp_train_noalloc: address of the partial-gradient array on device %d: %s",
                 dev, hipGetErrorString(e));
      return KP_E_DEVICE;
    }
    g_partials_ptr[dev] = static_cast<float*>(ptr);
  }
  *out = g_partials_ptr[dev];
  return KP_OK;
}
}  // namespace

extern "C" {

kp_status kp_mlp_pack(const float* dev_params, void* dev_packed, void* hip_stream) {
  if (!dev_params || !dev_packed || !aligned16(dev_packed)) return KP_E_ARG;
  if (launch_mlp_pack(dev_params, static_cast<uint4*>(dev_packed),
                      static_cast<hipStream_t>(hip_stream)) != hipSuccess)
    return KP_E_DEVICE;
  return KP_OK;
}

kp_status kp_mlp_forward(const void* dev_packed, const float* dev_x, int32_t rows, float* dev_out,
                         void* hip_stream) {
  if (rows < 0) return KP_E_ARG;
  if (rows == 0) return KP_OK;
  if (!dev_packed || !dev_x || !dev_out || !aligned16(dev_packed) || !aligned16(dev_x) ||
      !aligned16(dev_out))
    return KP_E_ARG;
  if (launch_mlp_forward(static_cast<const uint4*>(dev_packed), dev_x, rows, dev_out,
                         static_cast<hipStream_t>(hip_stream)) != hipSuccess)
    return KP_E_DEVICE;
  return KP_OK;
}

kp_status kp_mlp_grad(const void* dev_packed, const float* dev_x, const float* dev_t, int32_t n_rows,
                      int32_t n_ctrl, int32_t batch, uint64_t sample_key, int32_t step,
                      float* dev_partials, float* dev_loss, void* hip_stream) {
  if (!dev_packed || !dev_x || !dev_t || !dev_partials || !dev_loss || !aligned16(dev_packed) ||
      !aligned16(dev_x))
    return KP_E_ARG;
  if (n_rows < 1 || batch < 1 || n_ctrl < 1 || n_ctrl > 4 || step < 0) return KP_E_ARG;
  if (sample_key == 0 && batch > n_rows) return KP_E_ARG;
  if (launch_mlp_grad(static_cast<const uint4*>(dev_packed), dev_x, dev_t, n_rows, n_ctrl, batch,
                      sample_key, step, dev_partials, dev_loss,
                      static_cast<hipStream_t>(hip_stream)) != hipSuccess)
    return KP_E_DEVICE;
  return KP_OK;
}

kp_status kp_mlp_adam(float* dev_params, float* dev_m1, float* dev_m2, const float* dev_partials,
                      int32_t n_partials, int32_t step, float lr, float beta1, float beta2,
                      float eps, void* hip_stream) {
  if (!dev_params || !dev_m1 || !dev_m2 || !dev_partials || n_partials < 1 || step < 1)
    return KP_E_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
      !(lr >= 0.0f))
    return KP_E_ARG;
  const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
  const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
  if (!(bc1 > 0.0) || !(bc2 > 0.0)) return KP_E_ARG;
  if (launch_mlp_adam(dev_params, dev_m1, dev_m2, dev_partials, n_partials, lr, beta1, beta2, eps,
                      (float)(1.0 / bc1), (float)(1.0 / bc2),
                      static_cast<hipStream_t>(hip_stream)) != hipSuccess)
    return KP_E_DEVICE;
  return KP_OK;
}

kp_status kp_mlp_train(float* dev_params, float* dev_m1, float* dev_m2, void* dev_packed,
                       const float* dev_x, const float* dev_t, int32_t n_rows, int32_t n_ctrl,
                       int32_t batch, int32_t steps, int32_t step0, float lr, uint64_t sample_key,
                       float* dev_partials, float* dev_loss, void* hip_stream) {
  if (steps < 0 || step0 < 0 || sample_key == 0 || !dev_loss) return KP_E_ARG;
  const int32_t nb = (batch + KP_MLP_BLOCK_ROWS - 1) / KP_MLP_BLOCK_ROWS;
  for (int32_t k = 0; k < steps; ++k) {
    kp_status st = kp_mlp_pack(dev_params, dev_packed, hip_stream);
    if (st == KP_OK)
      st = kp_mlp_grad(dev_packed, dev_x, dev_t, n_rows, n_ctrl, batch, sample_key, step0 + k,
                       dev_partials, dev_loss + (size_t)k * nb, hip_stream);
    if (st == KP_OK)
      st = kp_mlp_adam(dev_params, dev_m1, dev_m2, dev_partials, nb, step0 + k + 1, lr, 0.9f,
                       0.999f, 1e-8f, hip_stream);
    if (st != KP_OK) return st;
  }
  return kp_mlp_pack(dev_params, dev_packed, hip_stream);
}

kp_status kp_mlp_train_noalloc(float* dev_params, float* dev_m1, float* dev_m2, void* dev_packed,
                               const float* dev_x, const float* dev_t, int32_t n_rows,
                               int32_t n_ctrl, int32_t batch, int32_t steps, int32_t step0,
                               float lr, uint64_t sample_key, float* dev_loss, void* hip_stream) {
  if (batch < 1 || batch > KP_MLP_STATIC_MAX_BATCH) {
    call_error("kp_mlp_train_noalloc: batch %d outside 1 .. %d (the static partial-gradient "
               "array holds %d partial gradients)", (int)batch, KP_MLP_STATIC_MAX_BATCH,
               kStaticPartials);
    return KP_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  float* partials = nullptr;
  const kp_status st = static_partials(s, &partials);
  if (st != KP_OK) return st;
  const kp_status r = kp_mlp_train(dev_params, dev_m1, dev_m2, dev_packed, dev_x, dev_t, n_rows,
                                   n_ctrl, batch, steps, step0, lr, sample_key, partials, dev_loss,
                                   hip_stream);
  if (r == KP_E_ARG) call_error("kp_mlp_train_noalloc: invalid argument (see kp_mlp_train)");
  else if (r != KP_OK) call_error("kp_mlp_train_noalloc: launch failed");
  return r;
}

kp_status kp_set_proposal(kp_problem* h, const void* dev_packed, float* dev_head, int64_t head_rows,
                          float mix) {
  if (!h) return KP_E_ARG;
  if (h->stage != 0) return fail(h, KP_E_ORDER, "kp_set_proposal in the middle of an iteration");
  // a uniform share 1 - mix > 0 keeps a positive density on all of U, which
  // the completeness argument (Sec. V, Theorem 1) needs
  if (!(mix >= 0.0f && mix < 1.0f)) return fail(h, KP_E_ARG, "mix must be in [0, 1)");
  const bool on = dev_packed != nullptr && mix > 0.0f;
  if (on) {
    if (!dev_head || head_rows < h->desc.node_cap || !aligned16(dev_packed) || !aligned16(dev_head))
      return fail(h, KP_E_ARG, "kp_set_proposal: head buffer must hold node_cap rows of 8 floats");
  }
  h->prm.mix_thr = on ? (unsigned long long)std::floor((double)mix * 4294967296.0) : 0ull;
  h->dev.mlp = on ? static_cast<const uint4*>(dev_packed) : nullptr;
  h->dev.head = on ? dev_head : nullptr;
  hipError_t e = upload_env(h);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "proposal upload");
  return KP_OK;
}

kp_status kp_log_path(kp_problem* h, int32_t node, float* dev_x, float* dev_t, int32_t cap_rows,
                      int32_t row0, int32_t* n_rows) {
  if (!h || !n_rows || !dev_x || !dev_t || cap_rows < 0 || row0 < 0) return KP_E_ARG;
  *n_rows = 0;
  int32_t len = 0;
  kp_status st = kp_get_path(h, node, nullptr, 0, &len);
  if (st != KP_OK) return st;
  const int32_t edges = len - 1;
  if (edges <= 0 || row0 >= cap_rows) return KP_OK;
  hipError_t e = launch_log_path(h->env_dev, dev_x, dev_t, cap_rows, row0, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "path logging");
  *n_rows = edges < cap_rows - row0 ? edges : cap_rows - row0;
  return KP_OK;
}

kp_status kp_log_tree_edges(kp_problem* h, float* dev_x, float* dev_t, int32_t cap_rows,
                            int32_t row0, int32_t* n_rows) {
  if (!h || !n_rows || !dev_x || !dev_t || cap_rows < 0 || row0 < 0) return KP_E_ARG;
  *n_rows = 0;
  if (h->stage != 0) return fail(h, KP_E_ORDER, "kp_log_tree_edges in the middle of an iteration");
  kp_status st = sync_ctl(h);
  if (st != KP_OK) return st;
  const int tiles = edge_tiles(h->hctl->N);
  // per-tile counts in the per-wave-tile count array of the V_U staging,
  // unused between iterations (it holds node_cap / 64 + 2 entries)
  if ((long long)tiles > (long long)h->desc.node_cap / 64 + 2)
    return fail(h, KP_E_ARG, "kp_log_tree_edges: tree too large for the count array");
  uint32_t* tcount = h->dev.scount;
  hipError_t e = launch_edge_count(h->env_dev, tiles, tcount, h->stream);
  if (e == hipSuccess)
    e = launch_edge_write(h->env_dev, tiles, tcount, dev_x, dev_t, cap_rows, row0, h->stream);
  std::vector<uint32_t> counts((size_t)tiles);
  if (e == hipSuccess && tiles > 0)
    e = hipMemcpyAsync(counts.data(), tcount, counts.size() * 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "tree edge logging");
  long long total = 0;
  for (uint32_t v : counts) total += v;
  const long long room = (long long)cap_rows - row0;
  *n_rows = (int32_t)(total < room ? total : (room > 0 ? room : 0));
  return KP_OK;
}

// ---------------------------------------------------------------------------
// batched planning
// ---------------------------------------------------------------------------
}  // extern "C"

struct kp_batch {
  std::vector<kp_problem*> P;
  const Env** table = nullptr;        // device: Env* of every problem
  BatchStatus* st_dev = nullptr;      // device: status of every problem
  BatchStatus* st_host = nullptr;     // pinned mirror
  hipStream_t stream = nullptr;       // the batch's own stream
  hipStream_t user_stream = nullptr;  // the problems' stream
  int dyn = 0, integ = 0;
  size_t lds_prop = 0;                // dynamic LDS of a propagate block: the largest problem's
  int region_blocks = 1;              // region blocks of a post grid row: the largest problem's
  size_t lds_queue = 0;               // dynamic LDS of a k_plan_queue workgroup: the largest problem's
  QueueCtl* q_ctl = nullptr;          // device: work queue of kp_batch_plan_queue
  int32_t* q_order = nullptr;
  QueueJob* q_jobs = nullptr;
  unsigned long long* q_t_end = nullptr;
  int32_t* q_ran = nullptr;
  int sym = 1;                        // every problem's state box is symmetric
  int learned = 0;                    // some problem has a learned proposal (set per plan)
  int prop_max = 1, node_max = 1;     // single-problem grid maxima
  kp_batch_config cfg{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
};

namespace {

size_t batch_table_bytes(int32_t n) { return align_up((size_t)n * sizeof(void*), kAlign); }

// Batch workspace: problem table, statuses, then the work queue of
// kp_batch_plan_queue (control word, order, budgets, end ticks, iterations).
struct BatchLayout {
  size_t table, status, qctl, order, jobs, t_end, ran, total;
};
BatchLayout batch_layout(int32_t n) {
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, kAlign);
    return o;
  };
  L.table = take((size_t)n * sizeof(void*));
  L.status = take((size_t)n * sizeof(BatchStatus));
  L.qctl = take(sizeof(QueueCtl));
  L.order = take((size_t)n * sizeof(int32_t));
  L.jobs = take((size_t)n * sizeof(QueueJob));
  L.t_end = take((size_t)n * sizeof(unsigned long long));
  L.ran = take((size_t)n * sizeof(int32_t));
  L.total = off;
  return L;
}

kp_status bfail(kp_batch* b, kp_status st, const std::string& msg) {
  if (b) b->err = msg;
  return st;
}
kp_status bhip(kp_batch* b, hipError_t e, const char* what) {
  return bfail(b, KP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void drop_graph(kp_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// one iteration for every problem: grids from per-problem bounds (capped)
hipError_t batch_iteration(kp_batch* b, long long lanes_ub, long long old_nodes_ub) {
  const int n = (int)b->P.size();
  if (b->learned) {
    // the proposal network of every problem that has one, before its expansion
    const long long rpb = mlp_head_rows_per_block();
    long long hb = (lanes_ub + rpb - 1) / rpb;
    const int cap = mlp_head_grid_max(b->P[0]->cu_count);
    hipError_t e = launch_mlp_head_batch(b->table, n, (int)(hb < cap ? hb : cap), b->stream);
    if (e != hipSuccess) return e;
  }
  long long t = (lanes_ub + 63) / 64;
  int gp = (int)(t < b->cfg.prop_blocks ? t : b->cfg.prop_blocks);
  if (gp < 1) gp = 1;
  gp = xcd_grid(gp, b->cfg.prop_blocks);
  t = (lanes_ub + kCommitBlock - 1) / kCommitBlock;
  const int nc = (int)(t < b->cfg.node_blocks ? t : b->cfg.node_blocks);
  t = (old_nodes_ub + kNodeTile - 1) / kNodeTile;
  int nn = (int)(t < b->cfg.node_blocks ? t : b->cfg.node_blocks);
  if (t > (long long)kChunkTilesMax * nn) nn = (int)((t + kChunkTilesMax - 1) / kChunkTilesMax);
  hipError_t e = launch_propagate_batch(b->dyn, b->integ, b->sym, b->table, n, b->lds_prop,
                                        gp < 1 ? 1 : gp, b->stream);
  if (e == hipSuccess) e = launch_post_batch(b->table, n, b->region_blocks, nc, nn, b->stream);
  return e;
}

kp_status batch_status(kp_batch* b) {
  const int n = (int)b->P.size();
  hipError_t e = launch_batch_status(b->table, n, b->st_dev, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->st_host, b->st_dev, (size_t)n * sizeof(BatchStatus), hipMemcpyDeviceToHost,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch status");
  for (int i = 0; i < n; ++i)
    if (b->st_host[i].err)
      return bfail(b, KP_E_DEVICE, "device check failed in problem " + std::to_string(i));
  return KP_OK;
}

// the graph of cfg.iters_per_sync iterations at the capped grids
kp_status batch_graph(kp_batch* b) {
  if (b->exec) return KP_OK;
  const long long big = (long long)1 << 40;
  // |T| is bounded by the largest node capacity (the node-set grid follows it)
  long long cap = 1;
  for (const kp_problem* h : b->P)
    if (h->desc.node_cap > cap) cap = h->desc.node_cap;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bhip(b, e, "graph capture");
  hipError_t le = hipSuccess;
  for (int k = 0; k < b->cfg.iters_per_sync && le == hipSuccess; ++k) le = batch_iteration(b, big, cap);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (le != hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return bhip(b, e, "graph instantiate");
  }
  return KP_OK;
}

}  // namespace

extern "C" {

size_t kp_batch_workspace_bytes(int32_t n) {
  if (n < 1) return 0;
  return batch_layout(n).total;
}

kp_status kp_batch_create(kp_problem* const* problems, int32_t n, void* dev_workspace, size_t bytes,
                          kp_batch** out) {
  if (!out) return KP_E_ARG;
  *out = nullptr;
  if (!problems || n < 1 || n > 65535 || !dev_workspace) return KP_E_ARG;
  if (bytes < kp_batch_workspace_bytes(n) || (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign))
    return KP_E_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    if (!problems[i]) return KP_E_ARG;
    if (problems[i]->desc.dynamics != problems[0]->desc.dynamics ||
        problems[i]->desc.integrator != problems[0]->desc.integrator)
      return KP_E_ARG;
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return KP_E_ARG;
  }
  kp_batch* b = new (std::nothrow) kp_batch();
  if (!b) return KP_E_ARG;
  b->P.assign(problems, problems + n);
  b->user_stream = problems[0]->stream;
  b->dyn = problems[0]->desc.dynamics;
  b->integ = problems[0]->desc.integrator;
  int prop_max = 1, node_max = 1;
  for (int i = 0; i < n; ++i) {
    const kp_problem* h = problems[i];
    if (h->lds_prop > b->lds_prop) b->lds_prop = h->lds_prop;
    if (post_region_blocks(h->R) > b->region_blocks) b->region_blocks = post_region_blocks(h->R);
    const size_t lq =
        queue_lds_bytes(h->desc.dynamics, h->desc.n_obstacles, (int)h->og.words.size());
    if (lq > b->lds_queue) b->lds_queue = lq;
    if (!h->prm.box_sym) b->sym = 0;
    if (h->grid_post_max > node_max) node_max = h->grid_post_max;
    if (h->grid_commit_max > node_max) node_max = h->grid_commit_max;
  }
  int bp = 1;
  occupancy_propagate(b->dyn, b->integ, b->sym, b->lds_prop, &bp);
  prop_max = bp * problems[0]->cu_count;
  b->prop_max = prop_max;
  b->node_max = node_max;
  b->cfg.iters_per_sync = 8;
  b->cfg.use_graph = 0;
  b->cfg.prop_blocks = prop_max;
  b->cfg.node_blocks = node_max;
  char* base = static_cast<char*>(dev_workspace);
  const BatchLayout BL = batch_layout(n);
  b->table = reinterpret_cast<const Env**>(base + BL.table);
  b->st_dev = reinterpret_cast<BatchStatus*>(base + BL.status);
  b->q_ctl = reinterpret_cast<QueueCtl*>(base + BL.qctl);
  b->q_order = reinterpret_cast<int32_t*>(base + BL.order);
  b->q_jobs = reinterpret_cast<QueueJob*>(base + BL.jobs);
  b->q_t_end = reinterpret_cast<unsigned long long*>(base + BL.t_end);
  b->q_ran = reinterpret_cast<int32_t*>(base + BL.ran);
  std::vector<const Env*> tab((size_t)n);
  for (int i = 0; i < n; ++i) tab[(size_t)i] = problems[i]->env_dev;
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&b->st_host), (size_t)n * sizeof(BatchStatus),
                      hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->table, tab.data(), (size_t)n * sizeof(void*), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    if (b->st_host) (void)hipHostFree(b->st_host);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return KP_E_DEVICE;
  }
  *out = b;
  return KP_OK;
}

kp_status kp_batch_set_config(kp_batch* b, const kp_batch_config* cfg) {
  if (!b || !cfg) return KP_E_ARG;
  if (cfg->iters_per_sync < 1 || cfg->iters_per_sync > 64 || cfg->prop_blocks < 1 ||
      cfg->node_blocks < 1 || (cfg->use_graph != 0 && cfg->use_graph != 1))
    return bfail(b, KP_E_ARG, "kp_batch_set_config: field out of range");
  b->cfg = *cfg;
  drop_graph(b);
  return KP_OK;
}

kp_status kp_batch_get_config(const kp_batch* b, kp_batch_config* cfg) {
  if (!b || !cfg) return KP_E_ARG;
  *cfg = b->cfg;
  return KP_OK;
}

kp_status kp_batch_plan(kp_batch* b, kp_plan_result* results, double* batch_ms) {
  if (!b || !results) return KP_E_ARG;
  const int n = (int)b->P.size();
  for (int i = 0; i < n; ++i)
    if (b->P[i]->stage != 0)
      return bfail(b, KP_E_ORDER, "problem " + std::to_string(i) + " is in the middle of an iteration");
  const auto t0 = std::chrono::steady_clock::now();
  auto now_ms = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  // order after the work already queued on the problems' stream
  hipError_t e = hipStreamSynchronize(b->user_stream);
  if (e != hipSuccess) return bhip(b, e, "problem stream");
  int learned = 0;
  for (int i = 0; i < n; ++i) {
    b->P[i]->ctl_fresh = false;
    if (b->P[i]->prm.mix_thr != 0ull) learned = 1;
  }
  if (learned != b->learned) {
    b->learned = learned;
    drop_graph(b);  // the captured iterations gain or lose the network pass
  }
  kp_status st = batch_status(b);
  if (st != KP_OK) return st;
  std::vector<uint32_t> it0((size_t)n);
  std::vector<int> active((size_t)n, 1), stopped_by_host((size_t)n, 0);
  std::vector<double> t_end((size_t)n, 0.0);
  std::vector<int> code((size_t)n, KP_TIMEOUT);
  for (int i = 0; i < n; ++i) it0[(size_t)i] = (uint32_t)b->st_host[i].iters_done;
  for (;;) {
    const double ms = now_ms();
    int n_active = 0;
    long long min_left = (long long)1 << 40, lanes_ub = 0, nodes_ub = 0, lanes_ub2 = 0, nodes_ub2 = 0;
    for (int i = 0; i < n; ++i) {
      if (!active[(size_t)i]) continue;
      const BatchStatus& s = b->st_host[i];
      const kp_problem* h = b->P[(size_t)i];
      const long long done_iters = (long long)(uint32_t)s.iters_done - it0[(size_t)i];
      if (s.done) {
        code[(size_t)i] = s.done;
      } else if (done_iters >= h->desc.max_iters || ms >= h->desc.t_max_ms) {
        // this problem's own budget: its kernels return at once from now on
        code[(size_t)i] = KP_TIMEOUT;
        stopped_by_host[(size_t)i] = 1;
        e = launch_set_done(h->env_dev, KP_TIMEOUT, b->stream);
        if (e != hipSuccess) return bhip(b, e, "budget stop");
      } else {
        ++n_active;
        const long long left = h->desc.max_iters - done_iters;
        if (left < min_left) min_left = left;
        if (s.lanes > lanes_ub) lanes_ub = s.lanes;
        if (s.N > nodes_ub) nodes_ub = s.N;
        const long long cap = h->desc.node_cap;
        if (cap - s.N > lanes_ub2) lanes_ub2 = cap - s.N;
        if (cap > nodes_ub2) nodes_ub2 = cap;
        continue;
      }
      active[(size_t)i] = 0;
      t_end[(size_t)i] = ms;
    }
    if (n_active == 0) break;
    long long len = b->cfg.iters_per_sync;
    if (len > min_left) len = min_left;
    if (b->cfg.use_graph && len == b->cfg.iters_per_sync) {
      if ((st = batch_graph(b)) != KP_OK) return st;
      e = hipGraphLaunch(b->exec, b->stream);
      if (e != hipSuccess) return bhip(b, e, "graph launch");
    } else {
      for (long long k = 0; k < len; ++k) {
        // exact sizes for the first iteration after a read, bounds after it
        e = batch_iteration(b, k == 0 ? lanes_ub : lanes_ub2, k == 0 ? nodes_ub : nodes_ub2);
        if (e != hipSuccess) return bhip(b, e, "batch launch");
      }
    }
    if ((st = batch_status(b)) != KP_OK) return st;
  }
  const double total = now_ms();
  for (int i = 0; i < n; ++i) {
    kp_problem* h = b->P[(size_t)i];
    const BatchStatus& s = b->st_host[i];
    if (stopped_by_host[(size_t)i]) {
      // a budget stop is the host's decision, as in kp_plan: the device state
      // stays resumable
      e = launch_set_done(h->env_dev, 0, b->stream);
      if (e != hipSuccess) return bhip(b, e, "budget resume");
    }
    kp_plan_result& r = results[i];
    std::memset(&r, 0, sizeof(r));
    r.status = code[(size_t)i];
    r.goal_id = (s.goal_id == kNoGoal) ? -1 : s.goal_id;
    r.iterations = (int32_t)((uint32_t)s.iters_done - it0[(size_t)i]);
    r.n_nodes = s.N;
    r.elapsed_ms = t_end[(size_t)i];
    r.lanes_total = s.lanes_total;
    r.valid_total = s.valid_total;
  }
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch end");
  for (int i = 0; i < n; ++i) {
    kp_plan_result& r = results[i];
    if (r.goal_id >= 0) {
      int32_t len = 0;
      if (kp_get_path(b->P[(size_t)i], r.goal_id, nullptr, 0, &len) == KP_OK) r.path_len = len;
    }
  }
  if (batch_ms) *batch_ms = total;
  return KP_OK;
}

// Switched off: the first GPU run of the persistent queue kernel did not
// finish (a batch of six small double-integrator problems), and no cause has
// been shown yet; every call is refused until one is.
constexpr bool kQueueEnabled = false;

kp_status kp_batch_plan_queue(kp_batch* b, kp_plan_result* results, double* batch_ms) {
  if (!b || !results) return KP_E_ARG;
  if (!kQueueEnabled)
    return bfail(b, KP_E_ARG,
                 "kp_batch_plan_queue is switched off: its first GPU run did not finish and the "
                 "cause is not yet known; use kp_batch_plan");
  const int n = (int)b->P.size();
  for (int i = 0; i < n; ++i) {
    if (b->P[i]->stage != 0)
      return bfail(b, KP_E_ORDER, "problem " + std::to_string(i) + " is in the middle of an iteration");
    if (b->P[i]->prm.mix_thr != 0ull)
      return bfail(b, KP_E_ARG, "kp_batch_plan_queue: problem " + std::to_string(i) +
                                    " has a learned proposal (use kp_batch_plan)");
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e = hipStreamSynchronize(b->user_stream);
  if (e != hipSuccess) return bhip(b, e, "problem stream");
  int dev = 0, rate_khz = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess || rate_khz <= 0) return bhip(b, e, "wall clock rate");
  // largest capacities first, so that the longest queries start at once
  std::vector<int32_t> order((size_t)n);
  for (int i = 0; i < n; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return b->P[(size_t)x]->desc.node_cap > b->P[(size_t)y]->desc.node_cap;
  });
  std::vector<QueueJob> jobs((size_t)n);
  for (int i = 0; i < n; ++i) {
    const kp_problem_desc& d = b->P[(size_t)i]->desc;
    jobs[(size_t)i].iters = d.max_iters;
    jobs[(size_t)i].pad = 0;
    const double t = (double)d.t_max_ms * (double)rate_khz;
    jobs[(size_t)i].ticks = (t > 0.0 && t < 1.8e19) ? (unsigned long long)t : 0ull;
  }
  QueueCtl qc{};
  qc.head = 0u;
  qc.t_start = ~0ull;
  e = hipMemcpyAsync(b->q_ctl, &qc, sizeof qc, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->q_order, order.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->q_jobs, jobs.data(), (size_t)n * sizeof(QueueJob), hipMemcpyHostToDevice,
                       b->stream);
  if (e != hipSuccess) return bhip(b, e, "queue upload");
  for (int i = 0; i < n; ++i) b->P[(size_t)i]->ctl_fresh = false;
  int bq = 1;
  occupancy_queue(b->dyn, b->integ, b->sym, b->lds_queue, &bq);
  const int slots = bq * b->P[0]->cu_count;
  e = launch_plan_queue(b->dyn, b->integ, b->sym, b->table, b->q_order, b->q_jobs, n, b->q_ctl,
                        b->q_t_end, b->q_ran, b->lds_queue, n < slots ? n : slots, b->stream);
  if (e != hipSuccess) return bhip(b, e, "queue launch");
  kp_status st = batch_status(b);
  if (st != KP_OK) return st;
  const double total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::vector<unsigned long long> t_end((size_t)n);
  std::vector<int32_t> ran((size_t)n);
  e = hipMemcpyAsync(&qc, b->q_ctl, sizeof qc, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t_end.data(), b->q_t_end, (size_t)n * 8, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ran.data(), b->q_ran, (size_t)n * 4, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "queue results");
  for (int i = 0; i < n; ++i) {
    const BatchStatus& s = b->st_host[i];
    if (s.err) return bfail(b, KP_E_DEVICE, "problem " + std::to_string(i) + ": device check failed");
    kp_plan_result& r = results[i];
    std::memset(&r, 0, sizeof(r));
    r.status = s.done ? s.done : KP_TIMEOUT;
    r.goal_id = (s.goal_id == kNoGoal) ? -1 : s.goal_id;
    r.iterations = ran[(size_t)i];
    r.n_nodes = s.N;
    // the problem's end on the device clock, from the first workgroup's start
    r.elapsed_ms = (t_end[(size_t)i] >= qc.t_start)
                       ? (double)(t_end[(size_t)i] - qc.t_start) / (double)rate_khz
                       : 0.0;
    r.lanes_total = s.lanes_total;
    r.valid_total = s.valid_total;
    if (r.goal_id >= 0) {
      int32_t len = 0;
      if (kp_get_path(b->P[(size_t)i], r.goal_id, nullptr, 0, &len) == KP_OK) r.path_len = len;
    }
  }
  if (batch_ms) *batch_ms = total;
  return KP_OK;
}

kp_status kp_batch_reset(kp_batch* b, const uint64_t* seeds) {
  if (!b || !seeds) return KP_E_ARG;
  // the set-up of every problem (as kp_reset) enqueued back to back, one wait
  for (size_t i = 0; i < b->P.size(); ++i) {
    kp_problem* h = b->P[i];
    h->desc.seed = seeds[i];
    h->prm.key0 = (uint32_t)seeds[i];
    h->prm.key1 = (uint32_t)(seeds[i] >> 32);
    h->ctl_fresh = false;
    hipError_t e = upload_env(h);
    if (e == hipSuccess) e = launch_zero(h->prm, h->dev, h->env_dev, h->stream);
    if (e == hipSuccess) {
      Vec12 xi;
      for (int k = 0; k < 12; ++k) xi.v[k] = h->desc.x_init[k];
      e = launch_root(h->env_dev, xi, h->stream);
    }
    if (e != hipSuccess) return bhip(b, e, "batch reset");
    kp_status st = do_frontier(h, 1);
    if (st != KP_OK) return bfail(b, st, h->err);
    h->stage = 0;
  }
  hipError_t e = hipStreamSynchronize(b->user_stream);
  if (e != hipSuccess) return bhip(b, e, "batch reset");
  return KP_OK;
}

kp_status kp_batch_destroy(kp_batch* b) {
  if (!b) return KP_E_ARG;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  (void)hipHostFree(b->st_host);
  (void)hipStreamDestroy(b->stream);
  delete b;
  return KP_OK;
}

const char* kp_batch_last_error(const kp_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"

// Host runtime of the voxel-EP library: grid object, brick map, device
// buffers, stimulus bookkeeping, the time-step drivers (explicit, implicit
// Euler PCG, bidomain with mixed-precision elliptic refinement) and the C ABI
// declared in include/ep.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/ep.h"
#include "ep_internal.h"
#include "ep_layout.h"

using namespace ep;

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
// Inner FP32 PCG of the elliptic refinement: relative reduction per outer
// step (asking one pass for more costs more iterations than it saves: FP32
// rounding of the operator limits what a pass gains in FP64 terms).
constexpr double kInnerRtol = 1e-3;

struct HostSync {          // pinned read-back block
  CGScalars cg;
  double sums[4];
  double qacc;
  int flags[4];
};

struct TimerPair {
  hipEvent_t a, b;
};

// kernel kinds that can be timed (ep_kernel_time ids): 0 the explicit step
// or one full CG iteration, 1 the CG set-up launch, 2 the bidomain parabolic
// stencil, 3 the FP64 elliptic residual, 4 CG launches that only detected
// convergence (or skipped after it)
// Initial guess of the implicit solve: polynomial extrapolation of the
// diffusion increments of at most kPredOrder past steps.  A ring of three
// increments (the newest written each step, two older ones read) and a
// ping-pong pair for the precomputed history term Q.
constexpr int kPredOrder = 4;
constexpr int kDRing = 3;

enum { KT_STENCIL = 0, KT_CGSETUP = 1, KT_PARABOLIC = 2, KT_RESID = 3, KT_CGTAIL = 4,
       KT_ADJ = 5, KT_INIT = 6, KT_UPDATE = 7, KT_COARSE = 8, KT_MULTI = 9, kTimers = 10 };
// explicit monodomain grids that fit one co-resident launch run at most this
// many steps per launch (a stimulus switching on or off ends a launch too)
constexpr int kMsMaxSteps = 4096;
// ... and only grids of at most this many bricks: the grid-wide barrier's
// cost grows with the workgroups that meet at it, and beyond about 128 of
// them one launch per step is faster (measured on MI355X: 64 bricks 3.3
// against 4.6 us per step in FP64; 152 bricks 4.5 against 4.8; 312 bricks
// 10.2 against 6.2)
constexpr int kMsMaxBricks = 128;
// the two-level preconditioner keeps at most this many aggregates (the dense
// inverse is kMaxAgg^2 FP32); aggregates are cubes of 1, 2, 4, ... bricks
constexpr int kMaxAgg = 8192;

}  // namespace

struct ep_grid_s {
  // description
  int n[3] = {0, 0, 0};
  double h = 0, dt = 0, theta = 0.5;
  ep_model model = EP_MONO;
  ep_prec prec = EP_F64;
  ep_diff diff = EP_DIFF_EXPLICIT;
  ep_ionic ionic{};
  double pcg_rtol = 1e-6, ell_rtol = 1e-8;
  int pcg_maxit = 50, ell_max_outer = 8, ell_inner_maxit = 2000;
  int jacobi_sweeps = 0;
  std::vector<ep_stim> stims;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  // layout
  int nbx = 0, nby = 0, nbz = 0, nb = 0;
  std::vector<int> brick_id;   // nbx*nby*nbz -> id or -1
  std::vector<int> brick_pos;  // id -> (bx, by, bz)
  std::vector<uint8_t> hmask;  // (nb+1)*512 brick layout
  int64_t n_tissue = 0;
  // bidomain bath: conducting body tissue around the heart, part of the
  // elliptic domain only.  hbody = heart or bath (== hmask without a bath).
  bool bath = false;
  double sig_bath = 0.0;
  std::vector<uint8_t> hbody;
  int64_t n_body = 0;
  int64_t nvox = 0;            // (nb+1)*512
  LaunchCfg L{};
  LaunchCfg Le{};              // the elliptic inner solve's kernels (larger persistent grid)
  int grid = 0;

  // device
  std::vector<void*> allocs;
  int64_t dev_bytes = 0;       // device bytes held now (256-byte granules)
  int64_t dev_peak = 0;        // the most held at once, call temporaries included
  int device = 0;              // the HIP device the grid's memory lives on
  // caller-owned arena (nullptr: the grid allocates)
  char* arena = nullptr;
  int64_t arena_bytes = 0, arena_used = 0;
  // call temporaries from a fixed device region instead (set only for the
  // duration of an allocation-free call; nullptr otherwise)
  char* temp_region = nullptr;
  size_t temp_cap = 0, temp_used = 0;
  bool adj_in_arena = false;
  int* d_nbr = nullptr;
  uint64_t* d_rowsn = nullptr;
  uint8_t* d_mask = nullptr;
  uint8_t* d_body = nullptr;   // elliptic domain (aliases d_mask without a bath)
  int* d_brick_id = nullptr;   // box brick -> brick id or -1 (device reads into box layout)
  void* d_v[2] = {nullptr, nullptr};
  void* d_w[2] = {nullptr, nullptr};
  void* d_tact = nullptr;
  void* d_jstim = nullptr;
  void* d_c[6] = {};          // monodomain D / intracellular, state precision
  double* d_ci64[6] = {};     // bidomain: A_i in FP64
  double* d_ck64[6] = {};     // bidomain: A_i + A_e in FP64
  float* d_ck32[6] = {};      // bidomain: A_i + A_e in FP32
  void* d_cr[2] = {nullptr, nullptr};  // implicit-step PCG vectors (state precision):
  void* d_cs[2] = {nullptr, nullptr};  // z = M^-1 r, p, t = M^-1 q, ping-pong pairs
  void* d_cw[2] = {nullptr, nullptr};
  void* d_dinv = nullptr;
  void* d_bprev[2] = {nullptr, nullptr};  // implicit solve: b of the last two steps
  void* d_dprev[kDRing] = {};  // ring of increments d = v_{k+1} - b_k
  void* d_q[2] = {nullptr, nullptr};  // history term of the next guess, ping-pong
  void* d_vs = nullptr;       // v* (bidomain; Jacobi implicit step: its right-hand side)
  double* d_phi = nullptr;
  double* d_phi_hist[3] = {};     // bidomain: ring of past solutions (extrapolated guess)
  int phi_sel = 0;                // ring slot of the next solution
  double* d_r64 = nullptr;
  float* d_x32 = nullptr;        // inner FP32 PCG of the elliptic refinement: x,
  float* d_r32[2] = {nullptr, nullptr};   // r and z,
  float* d_s32 = nullptr;                 // s = K p,
  float* d_w32 = nullptr;                 // w = K z,
  float* d_p32 = nullptr;                 // p
  // two-level preconditioner of the inner solve (aggregates of bricks)
  bool coarse_on = false;        // the coarse correction is applied
  int n_agg = 0, agg_edge = 1;   // aggregates; bricks per aggregate edge
  int agg_ld = 0;                // n_agg rounded up to a multiple of 4 (row pitch)
  int* d_agg = nullptr;          // nb + 1: brick -> aggregate (ghost -> n_agg)
  int* d_agg_ptr = nullptr;      // n_agg + 1: CSR of each aggregate's bricks
  int* d_agg_brk = nullptr;      // nb
  float* d_rb = nullptr;         // max(nb, agg_ld): brick sums of r (zero beyond nb)
  float* d_rc = nullptr;         // agg_ld: aggregate sums of r (zero beyond n_agg)
  float* d_cc = nullptr;         // n_agg + 1: coarse correction (last: 0, the ghost's)
  void* d_kinv = nullptr;        // n_agg x agg_ld: (Kc + s/n_agg)^-1 in FP16,
  float kinv_unscale = 1.0f;     //   scaled; times kinv_unscale gives the inverse
  float* d_dinvk = nullptr;
  void* d_d0[6] = {};         // explicit monodomain: unscaled voxel tensors (adjoint)
  void* d_adj = nullptr;      // adjoint work block (cached, grown on demand)
  size_t adj_cap = 0;
  double* d_partials = nullptr;   // per-block partial sums of one-brick-per-block launches
  double* d_cgp[2] = {nullptr, nullptr};  // persistent CG launches: ping-pong partials
  CGScalars* d_cg = nullptr;      // two solver-scalar records, ping-pong
  int* d_flags = nullptr;       // [0] non-finite v, [2] a multi-step barrier timed out
  // explicit monodomain, small grids: several steps per cooperative launch
  bool ms_on = false;
  int steps_per_launch = 0;    // caller's cap (0: kMsMaxSteps, 1: one step per launch)
  void* d_xms[2] = {nullptr, nullptr};  // v* exchange arrays (state precision)
  unsigned* d_bar = nullptr;   // grid-barrier arrival counter
  double* d_sums = nullptr;    // 8 doubles
  double* d_qacc = nullptr;
  double* d_qstep = nullptr;
  int64_t* d_stim_idx = nullptr;
  double* d_stim_val = nullptr;
  HostSync* hs = nullptr;      // pinned
  // CG status word: coherent pinned host memory the CG kernels write (one
  // 8-byte store per launch), polled by the host instead of a copy + wait
  volatile unsigned long long* hmirror = nullptr;
  unsigned long long* dmirror = nullptr;
  unsigned seq = 0;            // launch number of the last CG launch issued
  const CGScalars* last_cg = nullptr;   // device scalars of the last implicit solve

  // stimulus bookkeeping
  std::vector<int64_t> stim_u;                 // unique stimulated voxels (global index)
  std::vector<std::vector<int32_t>> stim_cov;  // per stimulus: positions in stim_u
  std::vector<double> stim_vals;
  std::vector<char> stim_active;
  bool stim_built = false;

  // state
  int cur = 0;
  int64_t step = 0;
  bool have_prev = false;      // d_v[1-cur] holds the previous step's v
  bool have_bprev = false;     // d_bprev[1-bsel] holds the previous step's b
  int pred_len = 0;            // consecutive implicit steps behind the current one
  int dsel = 0;                // ring slot of the next increment
  int phi_hist = 0;            // solved phi of past steps held in the ring (0..3)
  int bsel = 0;
  bool has_cond = false;
  bool nonfinite = false;
  int last_inner = 50;
  std::string err;

  // timing: bit k set = launches of kernel id k are bracketed by events,
  // in the steps whose index is a multiple of timing_period
  uint32_t timing = 0;
  int timing_period = 1;
  size_t tused[kTimers] = {};
  std::vector<TimerPair> tk[kTimers];
  double tms[kTimers] = {};
  int64_t tcount[kTimers] = {};
};

namespace {

// message of this thread's last failed ep_create_grid
std::string& create_error() {
  static thread_local std::string last;
  return last;
}

ep_status fail(ep_grid g, ep_status s, const std::string& msg) {
  if (g) g->err = msg;
  return s;
}

#define HIPCHK(g, expr)                                                            \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail((g), EP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t elem_size(ep_prec p) { return p == EP_F64 ? sizeof(double) : sizeof(float); }

template <typename P>
ep_status dalloc(ep_grid g, P** out, size_t bytes) {
  const size_t rb = (bytes + 255) & ~static_cast<size_t>(255);
  void* p = nullptr;
  if (g->arena) {
    if (g->arena_used + static_cast<int64_t>(rb) > g->arena_bytes)
      return fail(g, EP_ERR_OOM, "arena of " + std::to_string(g->arena_bytes) +
                                     " bytes is too small (" +
                                     std::to_string(g->arena_used + static_cast<int64_t>(rb)) +
                                     " bytes needed so far)");
    p = g->arena + g->arena_used;
  } else {
    hipError_t e = hipMalloc(&p, rb);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(g, EP_ERR_OOM, "hipMalloc of " + std::to_string(rb) + " bytes failed");
    }
  }
  hipError_t e = hipMemsetAsync(p, 0, rb, g->stream);
  if (e != hipSuccess) {
    if (!g->arena) (void)hipFree(p);
    return fail(g, EP_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  }
  if (g->arena) g->arena_used += static_cast<int64_t>(rb);
  else g->allocs.push_back(p);
  g->dev_bytes += static_cast<int64_t>(rb);
  g->dev_peak = std::max(g->dev_peak, g->dev_bytes);
  *out = static_cast<P*>(p);
  return EP_OK;
}

// Device temporaries of one call: carved from the call's fixed region (an
// allocation-free call) or the arena above their current use and given back
// when the call ends, or hipMalloc'd and freed.  The owner synchronises the
// grid's stream before they go.
struct Temps {
  ep_grid g;
  int64_t mark, held = 0;
  size_t region_mark;
  std::vector<void*> mine;
  explicit Temps(ep_grid gg) : g(gg), mark(gg->arena_used), region_mark(gg->temp_used) {}
  Temps(const Temps&) = delete;
  Temps& operator=(const Temps&) = delete;
  template <typename P>
  hipError_t get(P** out, size_t bytes) {
    const size_t rb = (bytes + 255) & ~static_cast<size_t>(255);
    void* p = nullptr;
    if (g->temp_region) {
      if (g->temp_used + rb > g->temp_cap) return hipErrorOutOfMemory;
      *out = reinterpret_cast<P*>(g->temp_region + g->temp_used);
      g->temp_used += rb;
      return hipSuccess;
    }
    if (g->arena) {
      if (g->arena_used + static_cast<int64_t>(rb) > g->arena_bytes) return hipErrorOutOfMemory;
      p = g->arena + g->arena_used;
      g->arena_used += static_cast<int64_t>(rb);
    } else {
      const hipError_t e = hipMalloc(&p, rb);
      if (e != hipSuccess) return e;
      mine.push_back(p);
    }
    held += static_cast<int64_t>(rb);
    g->dev_peak = std::max(g->dev_peak, g->dev_bytes + held);
    *out = static_cast<P*>(p);
    return hipSuccess;
  }
  ~Temps() {
    if (g->temp_region) g->temp_used = region_mark;
    if (g->arena) g->arena_used = mark;
    for (void* p : mine) (void)hipFree(p);
  }
};

#define TRY(expr)                     \
  do {                                \
    ep_status s_ = (expr);            \
    if (s_ != EP_OK) return s_;       \
  } while (0)

inline int64_t box_index(const ep_grid g, int x, int y, int z) {
  return (static_cast<int64_t>(x) * g->n[1] + y) * g->n[2] + z;
}

// global (brick-layout) index of box voxel (x, y, z), or -1 if its brick is absent
inline int64_t brick_index(const ep_grid g, int x, int y, int z) {
  const int id = g->brick_id[(static_cast<int64_t>(x >> 3) * g->nby + (y >> 3)) * g->nbz + (z >> 3)];
  if (id < 0) return -1;
  return static_cast<int64_t>(id) * kBV + (((x & 7) * 8 + (y & 7)) * 8 + (z & 7));
}

template <typename T>
CoefSet<T> coefs(const ep_grid g) {
  CoefSet<T> c;
  for (int k = 0; k < 6; ++k) c.c[k] = static_cast<const T*>(g->d_c[k]);
  return c;
}

CoefSet<double> cset64(double* const a[6]) {
  CoefSet<double> c;
  for (int k = 0; k < 6; ++k) c.c[k] = a[k];
  return c;
}

CoefSet<float> cset32(float* const a[6]) {
  CoefSet<float> c;
  for (int k = 0; k < 6; ++k) c.c[k] = a[k];
  return c;
}

template <typename T>
IonicT<T> ionic_t(const ep_grid g) {
  IonicT<T> p;
  p.inv_tau_in = static_cast<T>(1.0 / g->ionic.tau_in);
  p.inv_tau_out = static_cast<T>(1.0 / g->ionic.tau_out);
  p.inv_tau_open = static_cast<T>(1.0 / g->ionic.tau_open);
  p.inv_tau_close = static_cast<T>(1.0 / g->ionic.tau_close);
  p.v_gate = static_cast<T>(g->ionic.v_gate);
  p.exc = static_cast<T>(g->ionic.exc);
  return p;
}

// ---- timing ---------------------------------------------------------------
// launches of the current step are timed (every step, or a sample of them)
bool timing_step(const ep_grid g) {
  return g->timing_period <= 1 || g->step % g->timing_period == 0;
}

TimerPair* timer_begin(ep_grid g, int id) {
  if (!((g->timing >> id) & 1u) || !timing_step(g)) return nullptr;
  if (g->tused[id] == g->tk[id].size()) {
    TimerPair tp;
    // timing-only events: no system-scope fence (cache write-back and
    // invalidation) when they complete, which would otherwise stall the
    // launch that follows; the totals are read after a stream synchronize
    constexpr unsigned kTimingEvent = hipEventDisableSystemFence;
    if (hipEventCreateWithFlags(&tp.a, kTimingEvent) != hipSuccess ||
        hipEventCreateWithFlags(&tp.b, kTimingEvent) != hipSuccess)
      return nullptr;
    g->tk[id].push_back(tp);
  }
  TimerPair* tp = &g->tk[id][g->tused[id]++];
  (void)hipEventRecord(tp->a, g->stream);
  return tp;
}

void timer_end(ep_grid g, TimerPair* tp) {
  if (tp) (void)hipEventRecord(tp->b, g->stream);
}

// move the last `count` pairs recorded under `from` to `to`
void timer_retag(ep_grid g, int from, int to, int count) {
  if (!g->timing || !timing_step(g)) return;
  for (int i = 0; i < count && g->tused[from] > 0; ++i) {
    TimerPair tp = g->tk[from][--g->tused[from]];
    g->tk[from].erase(g->tk[from].begin() + static_cast<long>(g->tused[from]));
    if (g->tused[to] == g->tk[to].size()) {
      g->tk[to].push_back(tp);
    } else {
      g->tk[to].insert(g->tk[to].begin() + static_cast<long>(g->tused[to]), tp);
    }
    ++g->tused[to];
  }
}

void timer_collect(ep_grid g) {
  for (int id = 0; id < kTimers; ++id) {
    for (size_t i = 0; i < g->tused[id]; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, g->tk[id][i].a, g->tk[id][i].b) == hipSuccess) {
        g->tms[id] += ms;
        g->tcount[id] += 1;
      }
    }
    g->tused[id] = 0;
  }
}

// ---- stimulus -------------------------------------------------------------
ep_status build_stimuli(ep_grid g) {
  std::vector<int64_t> all;
  std::vector<std::vector<int64_t>> per(g->stims.size());
  for (size_t k = 0; k < g->stims.size(); ++k) {
    const ep_stim& s = g->stims[k];
    for (int x = std::max(0, s.lo[0]); x < std::min(g->n[0], s.hi[0]); ++x)
      for (int y = std::max(0, s.lo[1]); y < std::min(g->n[1], s.hi[1]); ++y)
        for (int z = std::max(0, s.lo[2]); z < std::min(g->n[2], s.hi[2]); ++z) {
          const int64_t gi = brick_index(g, x, y, z);
          if (gi < 0 || !g->hmask[gi]) continue;
          if (s.radius > 0.0) {
            const double dx = (x + 0.5) * g->h - s.center[0];
            const double dy = (y + 0.5) * g->h - s.center[1];
            const double dz = (z + 0.5) * g->h - s.center[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 <= s.radius * s.radius)) continue;
          }
          per[k].push_back(gi);
          all.push_back(gi);
        }
  }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  g->stim_u = all;
  g->stim_cov.assign(g->stims.size(), {});
  for (size_t k = 0; k < per.size(); ++k)
    for (int64_t gi : per[k])
      g->stim_cov[k].push_back(static_cast<int32_t>(
          std::lower_bound(all.begin(), all.end(), gi) - all.begin()));
  g->stim_vals.assign(all.size(), 0.0);
  g->stim_active.assign(g->stims.size(), 0);
  if (!all.empty()) {
    TRY(dalloc(g, &g->d_stim_idx, all.size() * sizeof(int64_t)));
    TRY(dalloc(g, &g->d_stim_val, all.size() * sizeof(double)));
    HIPCHK(g, hipMemcpyAsync(g->d_stim_idx, all.data(), all.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, g->stream));
  }
  g->stim_built = false;
  return EP_OK;
}

// Refresh the stimulus current field for step `step`; returns the field
// pointer, or nullptr when no stimulus is active.  With accum, the step's
// injected charge is added to the call's total by a launch here (the
// multi-step kernel adds it itself).
template <typename T>
ep_status update_stimulus(ep_grid g, int64_t step, const T** jstim, bool accum = true) {
  *jstim = nullptr;
  if (g->stim_u.empty()) return EP_OK;
  const double tn = static_cast<double>(step) * g->dt;
  bool any = false, changed = !g->stim_built;
  for (size_t k = 0; k < g->stims.size(); ++k) {
    const char a = (g->stims[k].t_on <= tn && tn < g->stims[k].t_off) ? 1 : 0;
    any = any || a;
    if (a != g->stim_active[k]) changed = true;
    g->stim_active[k] = a;
  }
  if (changed) {
    std::fill(g->stim_vals.begin(), g->stim_vals.end(), 0.0);
    for (size_t k = 0; k < g->stims.size(); ++k)
      if (g->stim_active[k])
        for (int32_t u : g->stim_cov[k]) g->stim_vals[u] += g->stims[k].amp;
    HIPCHK(g, hipMemcpyAsync(g->d_stim_val, g->stim_vals.data(),
                             g->stim_vals.size() * sizeof(double), hipMemcpyHostToDevice,
                             g->stream));
    // the copy reads pageable host memory; keep it alive until it has run
    HIPCHK(g, hipStreamSynchronize(g->stream));
    launch_stim_scatter<T>(g->stream, g->d_stim_idx, g->d_stim_val,
                           static_cast<int>(g->stim_u.size()), static_cast<T*>(g->d_jstim),
                           g->d_qstep);
    g->stim_built = true;
  }
  if (any) {
    if (accum) launch_q_accum(g->stream, g->d_qacc, g->d_qstep, g->dt * g->h * g->h * g->h);
    *jstim = static_cast<const T*>(g->d_jstim);
  }
  return EP_OK;
}

// Steps from `step` (at most `avail`) over which the set of active stimuli
// stays what it is at `step`.
int stim_run(const ep_grid g, int64_t step, int avail) {
  if (g->stim_u.empty()) return avail;
  auto on = [&](int64_t st, const ep_stim& s) {
    const double tn = static_cast<double>(st) * g->dt;
    return s.t_on <= tn && tn < s.t_off;
  };
  int m = 1;
  for (; m < avail; ++m) {
    bool same = true;
    for (const ep_stim& s : g->stims)
      if (on(step + m, s) != on(step, s)) {
        same = false;
        break;
      }
    if (!same) break;
  }
  return m;
}

// Wait until the CG status word shows launch `seq` (or a later one) and
// return it.  Spins on the coherent host word and makes no HIP call on the
// way: with a stream query every 1024 spins, the profiler showed a 6 us
// gap before every launch queued while the host waited.  Only after 5 ms
// without the word (far longer than any CG launch) does it check the
// stream, and should the stream have drained without the word (it never
// should), the device copy of the scalars (`dev`) is read instead.
ep_status wait_status(ep_grid g, unsigned seq, const CGScalars* dev, unsigned long long* out) {
  // launch numbers increase by one per CG launch (modulo 2^32); a later
  // launch's word serves too (`done` and the iteration count carry over)
  auto reached = [seq](unsigned long long v) {
    return static_cast<int>(static_cast<unsigned>(v >> 32) - seq) >= 0;
  };
  using clock = std::chrono::steady_clock;
  auto next_check = clock::now() + std::chrono::milliseconds(5);
  for (uint64_t spin = 1;; ++spin) {
    const unsigned long long v = *g->hmirror;
    if (reached(v)) {
      *out = v;
      return EP_OK;
    }
    if ((spin & 1023) == 0 && clock::now() >= next_check) {
      next_check = clock::now() + std::chrono::milliseconds(5);
      const hipError_t e = hipStreamQuery(g->stream);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return fail(g, EP_ERR_HIP, std::string("CG wait: ") + hipGetErrorString(e));
      const unsigned long long w = *g->hmirror;
      if (reached(w)) {
        *out = w;
        return EP_OK;
      }
      CGScalars c{};
      HIPCHK(g, hipMemcpy(&c, dev, sizeof(CGScalars), hipMemcpyDeviceToHost));
      *out = (static_cast<unsigned long long>(seq) << 32) |
             (static_cast<unsigned long long>(c.it & 0x3fffffff) << 2) |
             (static_cast<unsigned long long>(c.fail ? 1 : 0) << 1) |
             static_cast<unsigned long long>(c.done ? 1 : 0);
      return EP_OK;
    }
  }
}

// One-launch-per-iteration PCG solve after its init launch (scalars in
// d_cg[0], the init's (b.b, r.r) partials in d_cgp[0], z0 = M^-1 r0 in
// zb[0], x0 in x).  Launch k reads scalars / partials [k & 1] and writes
// [(k + 1) & 1]; it reads z_{k-1} from zb[(k - 1) & 1] (z_0 from zb[0]) and
// writes z_k to zb[k & 1], and p_k, t_k to pb[k & 1], tb[k & 1].  Each
// launch publishes its convergence test as it starts, so the host queues
// the next launch while the current one runs its stencil (launches 0 and 1
// go together); the launch that finds the solve done does only the last x
// update.  (Keeping two launches queued instead measured the same: the
// extra launch after the last update cost what it saved.)
template <typename T>
ep_status pcg_step_solve(ep_grid g, CoefSet<T> c, T c0, T c1, T* x, T* const zb[2],
                         T* const pb[2], T* const tb[2], int maxit, int* iters, bool* failed) {
  CGScalars* cg = g->d_cg;
  double* const* P = g->d_cgp;
  int n = 0;
  auto launch = [&](int k) {
    TimerPair* t0 = timer_begin(g, k == 0 ? KT_CGSETUP : KT_STENCIL);
    launch_pcg_step<T>(g->L, g->d_nbr, c, c0, c1, x, zb[k == 0 ? 0 : (k - 1) & 1], zb[k & 1],
                       pb[(k + 1) & 1], pb[k & 1], tb[(k + 1) & 1], tb[k & 1], k == 0 ? 1 : 0,
                       cg + (k & 1), cg + ((k + 1) & 1), P[k & 1], P[(k + 1) & 1], g->dmirror,
                       ++g->seq);
    timer_end(g, t0);
    ++n;
  };
  const int last = maxit + 1;      // launches 0 .. maxit + 1 at most
  int k = 0;
  launch(k++);
  launch(k++);
  const unsigned seq1 = g->seq;    // launch number of launch 1
  unsigned long long st = 0;
  for (int w = 1;; ++w) {
    if (w > 1 && k <= last) launch(k++);   // launch w, queued behind w - 1
    TRY(wait_status(g, seq1 + static_cast<unsigned>(w - 1), cg + ((w + 1) & 1), &st));
    if ((st & 1) || w >= last) break;
  }
  const int it = static_cast<int>((st >> 2) & 0x3fffffff);
  *iters = it;
  *failed = ((st >> 1) & 1) != 0 || !(st & 1);
  g->last_cg = cg + (k & 1);
  // launch 0 and launches 1..it-1 applied the operator; launch it (it >= 1)
  // did the last x update; launches after it found the solve done
  if (it == 0) {
    timer_retag(g, KT_STENCIL, KT_CGTAIL, n - 1);
    timer_retag(g, KT_CGSETUP, KT_CGTAIL, 1);
  } else {
    timer_retag(g, KT_STENCIL, KT_CGTAIL, n - 1 - it);
    timer_retag(g, KT_STENCIL, KT_UPDATE, 1);
  }
  return EP_OK;
}

// ---- step drivers -----------------------------------------------------------
template <typename T>
ep_status step_explicit(ep_grid g, const T* jstim) {
  const int c = g->cur, n = 1 - c;
  TimerPair* t0 = timer_begin(g, KT_STENCIL);
  launch_explicit<T>(g->L, g->d_nbr, coefs<T>(g), static_cast<const T*>(g->d_v[c]),
                     static_cast<const T*>(g->d_w[c]), jstim, static_cast<T*>(g->d_v[n]),
                     static_cast<T*>(g->d_w[n]), static_cast<T*>(g->d_tact), ionic_t<T>(g),
                     static_cast<T>(g->dt), static_cast<T>(g->theta),
                     static_cast<double>(g->step) * g->dt, g->d_flags, nullptr, 0);
  timer_end(g, t0);
  return EP_OK;
}

// Several explicit steps in one cooperative launch (grids whose bricks all
// fit on the device at once): as many as stay under one stimulus state, at
// most `avail`; *taken reports how many.
template <typename T>
ep_status step_explicit_ms(ep_grid g, int32_t avail, int32_t* taken) {
  const int cap = g->steps_per_launch > 1 ? g->steps_per_launch : kMsMaxSteps;
  const int m = std::min(stim_run(g, g->step, avail), cap);
  const T* jstim = nullptr;
  TRY(update_stimulus<T>(g, g->step, &jstim, /*accum=*/m < 2));
  if (m < 2) {
    TRY(step_explicit<T>(g, jstim));
    *taken = 1;
    return EP_OK;
  }
  const int c = g->cur, n = (g->cur + m) & 1;
  TimerPair* tp = timer_begin(g, KT_MULTI);
  const hipError_t e = launch_explicit_ms<T>(
      g->stream, g->nb, g->d_nbr, coefs<T>(g), static_cast<const T*>(g->d_v[c]),
      static_cast<const T*>(g->d_w[c]), jstim, static_cast<T*>(g->d_v[n]),
      static_cast<T*>(g->d_w[n]), static_cast<T*>(g->d_tact), static_cast<T*>(g->d_xms[0]),
      static_cast<T*>(g->d_xms[1]), ionic_t<T>(g), static_cast<T>(g->dt),
      static_cast<T>(g->theta), g->dt, static_cast<long long>(g->step), m, g->d_qacc,
      jstim ? g->d_qstep : nullptr, g->dt * g->h * g->h * g->h, g->d_bar, g->d_flags);
  timer_end(g, tp);
  HIPCHK(g, e);
  *taken = m;
  return EP_OK;
}

template <typename T>
ep_status step_explicit27(ep_grid g, const T* jstim) {
  const int c = g->cur, n = 1 - c;
  TimerPair* t0 = timer_begin(g, KT_STENCIL);
  launch_explicit27<T>(g->L, g->d_nbr, coefs<T>(g), static_cast<const T*>(g->d_v[c]),
                       static_cast<const T*>(g->d_w[c]), jstim, static_cast<T*>(g->d_v[n]),
                       static_cast<T*>(g->d_w[n]), static_cast<T*>(g->d_tact), ionic_t<T>(g),
                       static_cast<T>(g->dt), static_cast<T>(g->theta),
                       static_cast<double>(g->step) * g->dt, g->d_flags);
  timer_end(g, t0);
  return EP_OK;
}

template <typename T>
ep_status step_be(ep_grid g, const T* jstim, ep_step_info* acc) {
  const int c = g->cur, n = 1 - c;
  T* x = static_cast<T*>(g->d_v[n]);
  T* zv[2] = {static_cast<T*>(g->d_cr[0]), static_cast<T*>(g->d_cr[1])};
  T* pv[2] = {static_cast<T*>(g->d_cs[0]), static_cast<T*>(g->d_cs[1])};
  T* tv[2] = {static_cast<T*>(g->d_cw[0]), static_cast<T*>(g->d_cw[1])};
  // x (= d_v[n]) still holds the previous step's v: check its activation here
  // initial guess: polynomial through the last K = min(pred_len, 4) diffusion
  // increments; Q_n came from the previous step, Q_{n+1} is written now
  auto binom = [](int k, int j) {
    static const int t[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                                {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
    return (k >= 0 && k <= 4 && j >= 0 && j <= 4) ? t[k][j] : 0;
  };
  const int m = g->have_bprev ? g->pred_len : 0;
  const int K = std::min(kPredOrder, m);            // order of this step's guess
  const int K1 = std::min(kPredOrder, m + 1);       // order of the next step's guess
  const T* bprev = m >= 1 ? static_cast<const T*>(g->d_bprev[1 - g->bsel]) : nullptr;
  const T* qin = K >= 2 ? static_cast<const T*>(g->d_q[1 - g->bsel]) : nullptr;
  auto dback = [&](int k) {   // increment written k steps before this one's (k = 1, 2)
    return static_cast<const T*>(g->d_dprev[(g->dsel + kDRing - k) % kDRing]);
  };
  const T* d2 = m >= 2 ? dback(1) : nullptr;
  const T* d3 = m >= 3 ? dback(2) : nullptr;
  const T q2 = static_cast<T>(-binom(K1, 2)), q3 = static_cast<T>(binom(K1, 3));
  const T q4 = static_cast<T>(-binom(K1, 4));
  TimerPair* ti = timer_begin(g, KT_INIT);
  launch_be_init<T>(g->L, g->d_nbr, coefs<T>(g), static_cast<const T*>(g->d_v[c]),
                    static_cast<const T*>(g->d_w[c]), jstim, bprev, qin, static_cast<T>(K), d2,
                    d3, q2, q3, q4, static_cast<T*>(g->d_bprev[g->bsel]),
                    static_cast<T*>(g->d_dprev[g->dsel]), static_cast<T*>(g->d_q[g->bsel]),
                    x, static_cast<T*>(g->d_w[n]),
                    zv[0], ionic_t<T>(g), static_cast<T>(g->dt), static_cast<T*>(g->d_tact),
                    static_cast<T>(g->theta), static_cast<double>(g->step - 1) * g->dt,
                    g->have_prev ? 1 : 0, g->d_flags, g->d_cg, g->d_cgp[0],
                    g->pcg_rtol * g->pcg_rtol, g->pcg_maxit);
  timer_end(g, ti);
  int iters = 0;
  bool failed = false;
  TRY(pcg_step_solve<T>(g, coefs<T>(g), T(1), static_cast<T>(-g->dt), x, zv, pv, tv,
                        g->pcg_maxit, &iters, &failed));
  acc->cg_iters += iters;
  acc->cg_max = std::max(acc->cg_max, iters);
  if (failed) g->hs->flags[1] = 1;
  return EP_OK;
}

// Implicit Euler by the thesis's fixed number of Jacobi sweeps from the
// current potential: reaction into v*, then jacobi_sweeps sweeps of
// (I - dt A) v = v* starting from v*, the last one written to the new
// state, then the activation check of this step.
template <typename T>
ep_status step_jacobi(ep_grid g, const T* jstim, ep_step_info* acc) {
  const int c = g->cur, n = 1 - c;
  T* vs = static_cast<T*>(g->d_vs);
  T* out = static_cast<T*>(g->d_v[n]);
  T* scratch = static_cast<T*>(g->d_cr[0]);
  launch_ionic<T>(g->L, static_cast<const T*>(g->d_v[c]), static_cast<const T*>(g->d_w[c]), jstim,
                  vs, static_cast<T*>(g->d_w[n]), ionic_t<T>(g), static_cast<T>(g->dt));
  const int K = g->jacobi_sweeps;
  const T* in = vs;
  for (int j = 0; j < K; ++j) {
    // alternate so that sweep K - 1 writes the new state
    T* dst = ((K - 1 - j) % 2 == 0) ? out : scratch;
    TimerPair* t0 = timer_begin(g, KT_STENCIL);
    launch_jacobi<T>(g->L, g->d_nbr, coefs<T>(g), static_cast<T>(g->dt),
                     static_cast<const T*>(g->d_dinv), vs, in, dst);
    timer_end(g, t0);
    in = dst;
  }
  launch_activation<T>(g->L, static_cast<const T*>(g->d_v[c]), out, static_cast<T*>(g->d_tact),
                       static_cast<T>(g->dt), static_cast<T>(g->theta),
                       static_cast<double>(g->step) * g->dt, g->d_flags);
  acc->cg_iters += K;
  acc->cg_max = std::max(acc->cg_max, K);
  return EP_OK;
}

// Coarse operator of the two-level preconditioner: Kc = P^T K P over the
// aggregates (K = -(A_i + A_e), with a bath its body operator), from the FP64
// weights; every entry raised by s/n_agg with s = trace(K)/n_agg (each
// aggregate's summed diagonal, always positive, bounds its Kc entry), so the
// constants, K's null space, get an eigenvalue of K's own scale -- also when
// one aggregate makes Kc zero up to rounding; then its inverse in FP64 and an
// FP32 copy for the inner solve.
ep_status coarse_setup(ep_grid g, Temps& tmp) {
  const int n = g->n_agg;
  const size_t nn = static_cast<size_t>(n) * n;
  double *kb = nullptr, *kc = nullptr, *pinv = nullptr, *rp = nullptr, *cp = nullptr;
  const size_t panel = static_cast<size_t>(kGjPanel) * n * sizeof(double);
  if (tmp.get(&kb, static_cast<size_t>(g->nb) * kCoarseRow * sizeof(double)) != hipSuccess ||
      tmp.get(&kc, nn * sizeof(double)) != hipSuccess ||
      tmp.get(&pinv, static_cast<size_t>(kGjPanel) * kGjPanel * sizeof(double)) != hipSuccess ||
      tmp.get(&rp, panel) != hipSuccess || tmp.get(&cp, panel) != hipSuccess) {
    (void)hipGetLastError();
    return fail(g, EP_ERR_OOM, "no device memory for the coarse operator");
  }
  HIPCHK(g, hipMemsetAsync(kc, 0, nn * sizeof(double), g->stream));
  launch_coarse_setup(g->L, g->d_nbr, g->d_ck64, 0.0, -1.0, n, g->d_agg_ptr, g->d_agg_brk,
                      g->d_agg, kb, kc);
  std::vector<double> dg(std::max(n, g->nb));
  HIPCHK(g, hipMemcpy2DAsync(dg.data(), sizeof(double), kb + kNbr, kCoarseRow * sizeof(double),
                             sizeof(double), g->nb, hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  double trace = 0.0;
  for (int b = 0; b < g->nb; ++b) trace += dg[b];
  const double s = trace / n;
  if (!(s > 0.0) || !std::isfinite(s))
    return fail(g, EP_ERR_ARG, "the elliptic operator has no positive diagonal");
  launch_coarse_invert(g->stream, n, g->agg_ld, kc, s / n, pinv, rp, cp);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipMemcpy2DAsync(dg.data(), sizeof(double), kc, (n + 1) * sizeof(double),
                             sizeof(double), n, hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!(dg[i] > 0.0) || !std::isfinite(dg[i]))
      return fail(g, EP_ERR_HIP, "coarse operator inverse is not positive definite");
    dmax = std::max(dmax, dg[i]);
  }
  // an SPD matrix's largest entry lies on its diagonal: scale it to 2^14,
  // well inside FP16's range
  const double scale = 16384.0 / dmax;
  launch_coarse_pack(g->stream, n, g->agg_ld, kc, scale, g->d_kinv);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipStreamSynchronize(g->stream));
  g->kinv_unscale = static_cast<float>(dmax / 16384.0);
  return EP_OK;
}

// Inner solve of the elliptic refinement: PCG with the two-level
// preconditioner, one-reduction form, four launches per iteration (update;
// aggregate sums and coarse GEMV; apply).  The update launch publishes its
// convergence test as it starts; the host keeps `chunk` iterations queued
// ahead like the one-launch solvers.  Scalars ping-pong in d_cg[0/1]; the
// init's partials are in d_cgp[0], the apply's in d_cgp[1].
ep_status cg2_solve(ep_grid g, int maxit, int* chunk_hint, int* iters, bool* failed) {
  CGScalars* cg = g->d_cg;
  float* x = g->d_x32;
  float* r = g->d_r32[0];
  float* z = g->d_r32[1];
  float* p = g->d_p32;
  float* sv = g->d_s32;
  float* w = g->d_w32;
  const CoefSet<float> c = cset32(g->d_ck32);
  auto iter = [&](int j) {
    CGScalars* cout = cg + ((j + 1) & 1);
    TimerPair* tu = timer_begin(g, KT_UPDATE);
    launch_cg2_update(g->Le, x, r, p, sv, z, w, g->d_rb, j == 0 ? 0 : 1, cg + (j & 1), cout,
                      j == 0 ? g->d_cgp[0] : g->d_cgp[1], g->dmirror, ++g->seq);
    timer_end(g, tu);
    TimerPair* tc = timer_begin(g, KT_COARSE);
    if (g->coarse_on)
      launch_coarse_apply(g->stream, g->n_agg, g->agg_ld, g->agg_edge == 1, g->d_agg_ptr,
                          g->d_agg_brk, g->d_rb, g->d_rc, g->d_kinv, g->kinv_unscale, g->d_cc,
                          cout);
    timer_end(g, tc);
    TimerPair* ta = timer_begin(g, KT_STENCIL);
    launch_cg2_apply(g->Le, g->d_nbr, c, 0.0f, -1.0f, g->d_dinvk, r, g->d_cc, g->d_agg, z, w,
                     cout, g->d_cgp[1]);
    timer_end(g, ta);
  };
  int j = 0;
  iter(j++);
  int chunk = std::max(1, *chunk_hint);
  unsigned long long st = 0;
  for (;;) {
    for (int i = 0; i < chunk; ++i) iter(j++);
    TRY(wait_status(g, g->seq, cg + (j & 1), &st));
    if ((st & 1) || j >= maxit + 2) break;
    chunk = 1;
  }
  const int it = static_cast<int>((st >> 2) & 0x3fffffff);
  *iters = it;
  *failed = ((st >> 1) & 1) != 0 || !(st & 1);
  *chunk_hint = std::max(1, it);
  // applies after the update that found the solve done only returned
  timer_retag(g, KT_STENCIL, KT_CGTAIL, std::max(0, j - 1 - it));
  return EP_OK;
}

// Mixed-precision elliptic solve for phi given the source potential vsrc
// (FP64 refinement around FP32 Jacobi-PCG inner solves).
template <typename T>
ep_status elliptic(ep_grid g, const T* vsrc, double rtol, int max_outer, ep_solve_info* out) {
  const int G = g->grid;
  const double inv_count = 1.0 / static_cast<double>(g->n_body);
  int outer = 0;
  int64_t inner_total = 0;
  double relres = 0.0;
  bool corrected = false;
  bool ok = false;
  for (;;) {
    TimerPair* tr = timer_begin(g, KT_RESID);
    launch_resid64<T>(g->L, g->d_nbr, cset64(g->d_ci64), cset64(g->d_ck64), vsrc, g->d_phi,
                      g->d_r64, g->d_partials);
    timer_end(g, tr);
    launch_reduce_sum(g->stream, g->d_partials, G, 3, g->d_sums);
    HIPCHK(g, hipMemcpyAsync(g->hs->sums, g->d_sums, 3 * sizeof(double), hipMemcpyDeviceToHost,
                             g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    const double rr = g->hs->sums[0], bb = g->hs->sums[2];
    if (bb == 0.0) {   // zero source: phi = 0 in the gauge
      HIPCHK(g, hipMemsetAsync(g->d_phi, 0, static_cast<size_t>(g->nvox) * sizeof(double),
                               g->stream));
      relres = 0.0;
      corrected = false;
      ok = true;
      break;
    }
    relres = std::sqrt(rr / bb);
    if (relres <= rtol) { ok = true; break; }
    if (!std::isfinite(relres) || outer >= max_outer) break;
    const double tin = kInnerRtol;
    launch_inner_init(g->Le, g->d_r64, g->d_body, g->d_sums, inv_count, g->d_x32, g->d_r32[0],
                      g->d_cg, g->d_cgp[0], tin * tin, g->ell_inner_maxit);
    int iters = 0;
    bool failed = false;
    TRY(cg2_solve(g, g->ell_inner_maxit, &g->last_inner, &iters, &failed));
    inner_total += iters;
    if (failed && iters < g->ell_inner_maxit && g->coarse_on) {
      // Breakdown before the iteration limit: (r, M r) or the step's
      // curvature was not positive (or not finite), so the preconditioner
      // with the rounded coarse inverse is not positive definite on this
      // grid.  Drop the coarse correction for good and repeat the pass with
      // Jacobi alone; phi has not been touched.
      g->coarse_on = false;
      HIPCHK(g, hipMemsetAsync(g->d_cc, 0, static_cast<size_t>(g->n_agg + 1) * sizeof(float),
                               g->stream));
      continue;
    }
    launch_phi_correct(g->L, g->d_phi, g->d_x32, g->d_body, g->d_partials);
    launch_reduce_sum(g->stream, g->d_partials, G, 1, g->d_sums + 4);
    corrected = true;
    ++outer;
  }
  if (corrected) launch_phi_shift(g->L, g->d_phi, g->d_body, g->d_sums + 4, inv_count);
  if (out) {
    out->outer = outer;
    out->inner_iters = inner_total;
    out->relres = relres;
    out->precond = g->coarse_on ? 0 : 1;
  }
  return ok ? EP_OK : EP_ERR_NOCONV;
}

template <typename T>
ep_status step_bido(ep_grid g, const T* jstim, ep_step_info* acc) {
  const int c = g->cur, n = 1 - c;
  T* vs = static_cast<T*>(g->d_vs);
  launch_ionic<T>(g->L, static_cast<const T*>(g->d_v[c]), static_cast<const T*>(g->d_w[c]), jstim,
                  vs, static_cast<T*>(g->d_w[n]), ionic_t<T>(g), static_cast<T>(g->dt));
  // warm start: the last solution (still in d_phi), or the polynomial
  // through the last two or three
  auto hist = [&](int k) { return g->d_phi_hist[(g->phi_sel + 3 - k) % 3]; };   // k = 1 newest
  if (g->phi_hist >= 2)
    launch_phi_extrap(g->L, g->d_phi, hist(1), hist(2), hist(3), std::min(3, g->phi_hist));
  ep_solve_info si{};
  ep_status s = elliptic<T>(g, vs, g->ell_rtol, g->ell_max_outer, &si);
  HIPCHK(g, hipMemcpyAsync(g->d_phi_hist[g->phi_sel], g->d_phi,
                           static_cast<size_t>(g->nvox) * sizeof(double), hipMemcpyDeviceToDevice,
                           g->stream));
  g->phi_sel = (g->phi_sel + 1) % 3;
  g->phi_hist = std::min(3, g->phi_hist + 1);
  if (s == EP_ERR_NOCONV) g->hs->flags[1] = 1;
  else if (s != EP_OK) return s;
  acc->cg_iters += si.inner_iters;
  acc->cg_max = std::max<int32_t>(acc->cg_max, static_cast<int32_t>(si.inner_iters));
  acc->ell_outer += si.outer;
  acc->relres = si.relres;
  TimerPair* t0 = timer_begin(g, KT_PARABOLIC);
  launch_parabolic<T>(g->L, g->d_nbr, coefs<T>(g), vs, g->d_phi,
                      static_cast<const T*>(g->d_v[c]), static_cast<T*>(g->d_v[n]),
                      static_cast<T*>(g->d_tact), static_cast<T>(g->dt),
                      static_cast<T>(g->theta), static_cast<double>(g->step) * g->dt,
                      g->d_flags);
  timer_end(g, t0);
  return EP_OK;
}

template <typename T>
ep_status run_steps(ep_grid g, int32_t nsteps, ep_step_info* info) {
  ep_step_info acc{};
  HIPCHK(g, hipMemsetAsync(g->d_qacc, 0, sizeof(double), g->stream));
  g->hs->flags[1] = 0;
  for (int32_t s = 0; s < nsteps; ++s) {
    if (g->ms_on) {
      int32_t m = 1;
      TRY(step_explicit_ms<T>(g, nsteps - s, &m));
      g->cur = (g->cur + m) & 1;
      g->step += m;
      g->have_prev = true;
      s += m - 1;
      continue;
    }
    const T* jstim = nullptr;
    TRY(update_stimulus<T>(g, g->step, &jstim));
    if (g->model == EP_BIDO) {
      TRY(step_bido<T>(g, jstim, &acc));
    } else if (g->diff == EP_DIFF_BE_JACOBI) {
      TRY(step_jacobi<T>(g, jstim, &acc));
    } else if (g->diff == EP_DIFF_BE_PCG) {
      TRY(step_be<T>(g, jstim, &acc));
      g->bsel = 1 - g->bsel;
      if (g->have_bprev) g->dsel = (g->dsel + 1) % kDRing;   // d_{n-1} went into the ring
      g->pred_len = g->have_bprev ? g->pred_len + 1 : 1;
      g->have_bprev = true;
    } else if (g->diff == EP_DIFF_EXPLICIT27) {
      TRY(step_explicit27<T>(g, jstim));
    } else {
      TRY(step_explicit<T>(g, jstim));
    }
    g->cur = 1 - g->cur;
    g->step += 1;
    g->have_prev = true;
  }
  if (g->model == EP_MONO && g->diff == EP_DIFF_BE_PCG && nsteps > 0) {
    // activation of the last step (the next step's init would check it too;
    // the first-crossing rule makes that repeat harmless)
    launch_activation<T>(g->L, static_cast<const T*>(g->d_v[1 - g->cur]),
                         static_cast<const T*>(g->d_v[g->cur]), static_cast<T*>(g->d_tact),
                         static_cast<T>(g->dt), static_cast<T>(g->theta),
                         static_cast<double>(g->step - 1) * g->dt, g->d_flags);
  }
  const int noconv = g->hs->flags[1];
  launch_sum<T>(g->L, static_cast<const T*>(g->d_v[g->cur]), g->d_partials);
  launch_reduce_sum(g->stream, g->d_partials, g->grid, 1, g->d_sums + 6);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipMemcpyAsync(g->hs->sums + 3, g->d_sums + 6, sizeof(double), hipMemcpyDeviceToHost,
                           g->stream));
  HIPCHK(g, hipMemcpyAsync(&g->hs->qacc, g->d_qacc, sizeof(double), hipMemcpyDeviceToHost,
                           g->stream));
  HIPCHK(g, hipMemcpyAsync(g->hs->flags, g->d_flags, 4 * sizeof(int), hipMemcpyDeviceToHost,
                           g->stream));
  const bool be = g->model == EP_MONO && g->diff == EP_DIFF_BE_PCG && nsteps > 0 && g->last_cg;
  if (be)
    HIPCHK(g, hipMemcpyAsync(&g->hs->cg, g->last_cg, sizeof(CGScalars), hipMemcpyDeviceToHost,
                             g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  if (be && g->hs->cg.bb > 0) acc.relres = std::sqrt(g->hs->cg.rr / g->hs->cg.bb);
  timer_collect(g);
  const double h3 = g->h * g->h * g->h;
  acc.steps = nsteps;
  acc.step = g->step;
  acc.t = static_cast<double>(g->step) * g->dt;
  acc.q_stim = g->hs->qacc;
  acc.mass = h3 * g->hs->sums[3];
  if (info) *info = acc;
  if (g->hs->flags[2]) {
    // cannot happen with a cooperative launch; should it, the grid goes back
    // to one launch per step and the state of this call is not to be used
    g->ms_on = false;
    g->hs->flags[2] = 0;
    HIPCHK(g, hipMemsetAsync(g->d_flags + 2, 0, sizeof(int), g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return fail(g, EP_ERR_HIP, "a grid-wide barrier of the multi-step kernel timed out");
  }
  if (g->hs->flags[0]) g->nonfinite = true;
  if (g->nonfinite) return fail(g, EP_ERR_NONFINITE, "non-finite potential");
  if (noconv) return fail(g, EP_ERR_NOCONV, "a linear solve hit its iteration limit");
  return EP_OK;
}

// ---- adjoint of the explicit monodomain run (checkpointed) ------------------
// Forward: nsteps explicit steps from the current state with a fresh T_act,
// recording each voxel's crossing step and, every K steps, a checkpoint
// (v, w at the segment start and v one step earlier).  Backward: per segment,
// last first, the segment's states are recomputed from its checkpoint (the
// forward kernel is deterministic, so they are bitwise the forward's) and the
// adjoint kernel runs once per step, last step first.
template <typename T>
ep_status adjoint_impl(ep_grid g, int32_t nsteps, int32_t K, const double* tstar_box,
                       double* loss, double* grad_box, int64_t* n_used) {
  const int64_t nv = g->nvox;
  const size_t vb = static_cast<size_t>(nv) * sizeof(T);
  // without grad_box only the forward run and the loss: no checkpoints
  const bool want_grad = grad_box != nullptr;
  const int S = want_grad ? (nsteps + K - 1) / K : 0;
  // work block: grad (FP64), cross, T*, lv/lw ping-pong, checkpoints, segment
  const size_t n_arr =
      want_grad ? 1 + 4 + 3 * static_cast<size_t>(S) + 2 * (static_cast<size_t>(K) + 1) : 1;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t need =
      (want_grad ? al(nv * sizeof(double)) : 0) + al(nv * sizeof(int)) + n_arr * al(vb);
  if (need > g->adj_cap) {
    if (g->d_adj && !g->adj_in_arena) {
      HIPCHK(g, hipStreamSynchronize(g->stream));
      (void)hipFree(g->d_adj);
      g->dev_bytes -= static_cast<int64_t>(g->adj_cap);
    }
    g->d_adj = nullptr;
    g->adj_cap = 0;
    if (g->arena) {
      // carved for good: a later, larger call takes a new block above it
      const int64_t rb = static_cast<int64_t>(al(need));
      if (g->arena_used + rb > g->arena_bytes)
        return fail(g, EP_ERR_OOM, "adjoint work block of " + std::to_string(need) +
                                       " bytes does not fit in the arena");
      g->d_adj = g->arena + g->arena_used;
      g->arena_used += rb;
      g->adj_in_arena = true;
    } else if (hipMalloc(&g->d_adj, need) != hipSuccess) {
      (void)hipGetLastError();
      g->d_adj = nullptr;
      return fail(g, EP_ERR_OOM, "adjoint work block of " + std::to_string(need) +
                                     " bytes does not fit; raise ckpt_every or lower nsteps");
    }
    g->adj_cap = need;
    g->dev_bytes += static_cast<int64_t>(al(need));
    g->dev_peak = std::max(g->dev_peak, g->dev_bytes);
  }
  char* base = static_cast<char*>(g->d_adj);
  size_t off = 0;
  auto take = [&](size_t b) {
    void* p = base + off;
    off += al(b);
    return p;
  };
  double* d_grad = want_grad ? static_cast<double*>(take(nv * sizeof(double))) : nullptr;
  int* d_cross = static_cast<int*>(take(nv * sizeof(int)));
  T* d_tstar = static_cast<T*>(take(vb));
  T* lv[2] = {nullptr, nullptr};
  T* lw[2] = {nullptr, nullptr};
  std::vector<T*> ck_v(S), ck_w(S), ck_vp(S), seg_v, seg_w;
  if (want_grad) {
    for (int i = 0; i < 2; ++i) {
      lv[i] = static_cast<T*>(take(vb));
      lw[i] = static_cast<T*>(take(vb));
    }
    for (int c = 0; c < S; ++c) {
      ck_v[c] = static_cast<T*>(take(vb));
      ck_w[c] = static_cast<T*>(take(vb));
      ck_vp[c] = static_cast<T*>(take(vb));
    }
    seg_v.resize(K + 1);
    seg_w.resize(K + 1);
    for (int i = 0; i <= K; ++i) {
      seg_v[i] = static_cast<T*>(take(vb));
      seg_w[i] = static_cast<T*>(take(vb));
    }
  }

  // targets to brick layout (non-finite = no target; non-tissue = no target)
  {
    std::vector<T> ht(nv, std::numeric_limits<T>::infinity());
    parallel_for(g->n[0], [&](int64_t xx) {
      const int x = static_cast<int>(xx);
      for (int y = 0; y < g->n[1]; ++y)
        for (int z = 0; z < g->n[2]; ++z) {
          const int64_t gi = brick_index(g, x, y, z);
          if (gi < 0 || !g->hmask[gi]) continue;
          const double t = tstar_box[box_index(g, x, y, z)];
          ht[gi] = std::isfinite(t) ? static_cast<T>(t) : std::numeric_limits<T>::infinity();
        }
    });
    HIPCHK(g, hipMemcpyAsync(d_tstar, ht.data(), vb, hipMemcpyHostToDevice, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
  }
  if (want_grad) HIPCHK(g, hipMemsetAsync(d_grad, 0, nv * sizeof(double), g->stream));
  HIPCHK(g, hipMemsetAsync(d_cross, 0xff, nv * sizeof(int), g->stream));  // -1
  {
    std::vector<T> inf(nv, std::numeric_limits<T>::infinity());
    HIPCHK(g, hipMemcpyAsync(g->d_tact, inf.data(), vb, hipMemcpyHostToDevice, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
  }
  HIPCHK(g, hipMemsetAsync(g->d_qacc, 0, sizeof(double), g->stream));

  const CoefSet<T> c = coefs<T>(g);
  CoefSet<T> d0;
  for (int k = 0; k < 6; ++k) d0.c[k] = static_cast<const T*>(g->d_d0[k]);
  const IonicT<T> ion = ionic_t<T>(g);
  const T dt = static_cast<T>(g->dt), theta = static_cast<T>(g->theta);
  const int64_t step0 = g->step;
  T* tact = static_cast<T*>(g->d_tact);

  // forward
  for (int32_t s = 0; s < nsteps; ++s) {
    const int cu = g->cur, nx = 1 - cu;
    if (want_grad && s % K == 0) {
      const int ci = s / K;
      HIPCHK(g, hipMemcpyAsync(ck_v[ci], g->d_v[cu], vb, hipMemcpyDeviceToDevice, g->stream));
      HIPCHK(g, hipMemcpyAsync(ck_w[ci], g->d_w[cu], vb, hipMemcpyDeviceToDevice, g->stream));
      if (s > 0)
        HIPCHK(g, hipMemcpyAsync(ck_vp[ci], g->d_v[nx], vb, hipMemcpyDeviceToDevice, g->stream));
    }
    const T* jstim = nullptr;
    TRY(update_stimulus<T>(g, step0 + s, &jstim));
    TimerPair* t0 = timer_begin(g, KT_STENCIL);
    launch_explicit<T>(g->L, g->d_nbr, c, static_cast<const T*>(g->d_v[cu]),
                       static_cast<const T*>(g->d_w[cu]), jstim, static_cast<T*>(g->d_v[nx]),
                       static_cast<T*>(g->d_w[nx]), tact, ion, dt, theta,
                       static_cast<double>(step0 + s) * g->dt, g->d_flags, d_cross, s);
    timer_end(g, t0);
    g->cur = nx;
    g->step += 1;
    g->have_prev = true;
  }
  HIPCHK(g, hipGetLastError());

  // loss over voxels activated in the run with a finite target
  launch_loss<T>(g->L, g->d_mask, d_cross, tact, d_tstar, g->d_partials);
  launch_reduce_sum(g->stream, g->d_partials, g->grid, 2, g->d_sums + 4);
  HIPCHK(g, hipMemcpyAsync(g->hs->sums, g->d_sums + 4, 2 * sizeof(double),
                           hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipMemcpyAsync(g->hs->flags, g->d_flags, sizeof(int), hipMemcpyDeviceToHost,
                           g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  if (g->hs->flags[0]) {
    g->nonfinite = true;
    return fail(g, EP_ERR_NONFINITE, "non-finite potential in the forward run");
  }
  *loss = g->hs->sums[0];
  *n_used = static_cast<int64_t>(g->hs->sums[1] + 0.5);
  if (!want_grad) {
    timer_collect(g);
    return EP_OK;
  }

  // backward: lambda_N from the crossings of the last step
  int a = 0;
  launch_adj_init<T>(g->L, g->d_mask, static_cast<const T*>(g->d_v[g->cur]),
                     static_cast<const T*>(g->d_v[1 - g->cur]), d_cross, tact, d_tstar, lv[0],
                     lw[0], dt, theta, nsteps - 1);
  const T inv_h2 = static_cast<T>(1.0 / (g->h * g->h));
  for (int ci = S - 1; ci >= 0; --ci) {
    const int s0 = ci * K, s1 = std::min(nsteps, s0 + K);
    HIPCHK(g, hipMemcpyAsync(seg_v[0], ck_v[ci], vb, hipMemcpyDeviceToDevice, g->stream));
    HIPCHK(g, hipMemcpyAsync(seg_w[0], ck_w[ci], vb, hipMemcpyDeviceToDevice, g->stream));
    // recompute v_{s0+1..s1}, w_{s0+1..s1}; T_act is already set wherever a
    // crossing happens, so the kernel leaves it (and the crossing steps) alone
    for (int s = s0; s < s1; ++s) {
      const T* jstim = nullptr;
      TRY(update_stimulus<T>(g, step0 + s, &jstim));
      const int i = s - s0;
      TimerPair* t0 = timer_begin(g, KT_STENCIL);
      launch_explicit<T>(g->L, g->d_nbr, c, seg_v[i], seg_w[i], jstim, seg_v[i + 1],
                         seg_w[i + 1], tact, ion, dt, theta,
                         static_cast<double>(step0 + s) * g->dt, g->d_flags, nullptr, 0);
      timer_end(g, t0);
    }
    for (int s = s1 - 1; s >= s0; --s) {
      const T* jstim = nullptr;
      TRY(update_stimulus<T>(g, step0 + s, &jstim));
      const int i = s - s0;
      const T* vprev = (i > 0) ? seg_v[i - 1] : (ci > 0 ? ck_vp[ci] : nullptr);
      TimerPair* t0 = timer_begin(g, KT_ADJ);
      launch_adj_step<T>(g->L, g->d_nbr, c, d0, g->d_mask, lv[a], lw[a], lv[1 - a], lw[1 - a],
                         seg_v[i], seg_w[i], jstim, seg_v[i + 1], vprev, d_cross, tact, d_tstar,
                         d_grad, ion, dt, theta, inv_h2, s);
      timer_end(g, t0);
      a = 1 - a;
    }
  }
  HIPCHK(g, hipGetLastError());
  std::vector<double> hg(nv);
  HIPCHK(g, hipMemcpyAsync(hg.data(), d_grad, nv * sizeof(double), hipMemcpyDeviceToHost,
                           g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  timer_collect(g);
  parallel_for(g->n[0], [&](int64_t xx) {
    const int x = static_cast<int>(xx);
    for (int y = 0; y < g->n[1]; ++y)
      for (int z = 0; z < g->n[2]; ++z) {
        const int64_t gi = brick_index(g, x, y, z);
        grad_box[box_index(g, x, y, z)] = (gi < 0 || !g->hmask[gi]) ? 0.0 : hg[gi];
      }
  });
  return EP_OK;
}

// dt * lambda_max(-A) < 2: accept on the Gershgorin bound, else estimate
// lambda_max by 200 power iterations and accept below 2 / 1.02.
ep_status check_explicit_stability(ep_grid g, double* const c64[6]) {
  const int G = g->grid;
  launch_block_max(g->L, g->d_nbr, cset64(c64), g->d_partials);
  std::vector<double> part(G);
  HIPCHK(g, hipMemcpyAsync(part.data(), g->d_partials, G * sizeof(double), hipMemcpyDeviceToHost,
                           g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  double gersh = 0.0;
  for (double v : part) gersh = (v > gersh || std::isnan(v)) ? v : gersh;
  if (std::isnan(gersh)) return fail(g, EP_ERR_ARG, "non-finite diffusion coefficients");
  if (g->dt * gersh < 2.0) return EP_OK;
  double *x = nullptr, *y = nullptr;
  const size_t bytes = static_cast<size_t>(g->nvox) * sizeof(double);
  Temps tmp(g);
  if (tmp.get(&x, bytes) != hipSuccess || tmp.get(&y, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(g, EP_ERR_OOM, "no device memory for the stability estimate");
  }
  std::vector<double> hx(g->nvox, 0.0);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (int64_t i = 0; i < g->nb * (int64_t)kBV; ++i) {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    hx[i] = g->hmask[i] ? (static_cast<double>(st >> 11) * 0x1.0p-53 - 0.5) : 0.0;
  }
  HIPCHK(g, hipMemcpyAsync(x, hx.data(), bytes, hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  double lam = 0.0;
  for (int it = 0; it < 200; ++it) {
    launch_apply<double>(g->L, g->d_nbr, cset64(c64), x, y, g->d_partials);
    launch_reduce_sum(g->stream, g->d_partials, G, 2, g->d_sums);
    launch_scale(g->L, x, y, g->d_sums);
  }
  HIPCHK(g, hipMemcpyAsync(g->hs->sums, g->d_sums, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  // x was unit before the last apply: lambda ~ |x . A x|
  lam = std::fabs(g->hs->sums[1]);
  if (!(g->dt * lam * 1.02 < 2.0)) {
    char buf[160];
    snprintf(buf, sizeof buf, "explicit diffusion unstable: dt*lambda_max(-A) ~ %.3f >= 2",
             g->dt * lam);
    return fail(g, EP_ERR_ARG, buf);
  }
  return EP_OK;
}

// 6-connected components of the tissue (host BFS), for the bidomain gauge
int64_t tissue_components(const std::vector<uint8_t>& m, const int n[3]) {
  const int64_t N = static_cast<int64_t>(n[0]) * n[1] * n[2];
  std::vector<uint8_t> seen(N, 0);
  std::vector<int64_t> stack;
  int64_t comps = 0;
  for (int64_t s = 0; s < N; ++s) {
    if (!m[s] || seen[s]) continue;
    ++comps;
    seen[s] = 1;
    stack.push_back(s);
    while (!stack.empty()) {
      const int64_t p = stack.back();
      stack.pop_back();
      const int z = static_cast<int>(p % n[2]);
      const int y = static_cast<int>((p / n[2]) % n[1]);
      const int x = static_cast<int>(p / (static_cast<int64_t>(n[1]) * n[2]));
      const int c[3] = {x, y, z};
      for (int d = 0; d < 3; ++d)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          int q3[3] = {c[0], c[1], c[2]};
          q3[d] += sgn;
          if (q3[d] < 0 || q3[d] >= n[d]) continue;
          const int64_t q = (static_cast<int64_t>(q3[0]) * n[1] + q3[1]) * n[2] + q3[2];
          if (m[q] && !seen[q]) { seen[q] = 1; stack.push_back(q); }
        }
    }
  }
  return comps;
}

ep_status create_impl(const ep_grid_desc* d, ep_grid g) {
  HIPCHK(g, hipGetDevice(&g->device));
  for (int k = 0; k < 3; ++k)
    if (d->n[k] < 1 || d->n[k] > 4096) return fail(g, EP_ERR_ARG, "n must be in [1, 4096]");
  if (!(d->h > 0) || !std::isfinite(d->h)) return fail(g, EP_ERR_ARG, "h must be > 0");
  if (!(d->dt > 0) || !std::isfinite(d->dt)) return fail(g, EP_ERR_ARG, "dt must be > 0");
  if (d->model != EP_MONO && d->model != EP_BIDO) return fail(g, EP_ERR_ARG, "bad model");
  if (d->prec != EP_F64 && d->prec != EP_F32) return fail(g, EP_ERR_ARG, "bad precision");
  if (d->diff != EP_DIFF_EXPLICIT && d->diff != EP_DIFF_BE_PCG && d->diff != EP_DIFF_BE_JACOBI &&
      d->diff != EP_DIFF_EXPLICIT27)
    return fail(g, EP_ERR_ARG, "bad diffusion scheme");
  if (d->diff == EP_DIFF_BE_JACOBI && d->jacobi_sweeps < 1)
    return fail(g, EP_ERR_ARG, "jacobi_sweeps >= 1 required");
  if (d->model == EP_BIDO && d->diff != EP_DIFF_EXPLICIT)
    return fail(g, EP_ERR_UNSUPPORTED, "bidomain takes the explicit 19-point step only");
  if (d->n_stim < 0 || (d->n_stim > 0 && !d->stim)) return fail(g, EP_ERR_ARG, "bad stimuli");
  if (d->bath && d->model != EP_BIDO)
    return fail(g, EP_ERR_UNSUPPORTED, "a bath belongs to the bidomain elliptic solve");
  if (d->bath && (!(d->sig_bath > 0) || !std::isfinite(d->sig_bath)))
    return fail(g, EP_ERR_ARG, "sig_bath must be finite and > 0");
  if (d->arena && (d->arena_bytes <= 0 || reinterpret_cast<uintptr_t>(d->arena) % 256 != 0))
    return fail(g, EP_ERR_ARG, "arena must be 256-byte aligned with arena_bytes > 0");
  const ep_ionic& io = d->ionic;
  if (!(io.tau_in > 0) || !(io.tau_out > 0) || !(io.tau_open > 0) || !(io.tau_close > 0) ||
      !std::isfinite(io.v_gate) || !std::isfinite(io.exc) || io.exc < 0)
    return fail(g, EP_ERR_ARG, "ionic time constants must be > 0 and exc >= 0");
  if (!(d->act_threshold > 0 && d->act_threshold < 1))
    return fail(g, EP_ERR_ARG, "act_threshold must be in (0, 1)");
  if (d->diff == EP_DIFF_BE_PCG && (!(d->pcg_rtol > 0) || d->pcg_maxit < 1))
    return fail(g, EP_ERR_ARG, "pcg_rtol > 0 and pcg_maxit >= 1 required");
  if (d->model == EP_BIDO &&
      (!(d->ell_rtol > 0) || d->ell_max_outer < 1 || d->ell_inner_maxit < 1))
    return fail(g, EP_ERR_ARG, "ell_rtol > 0, ell_max_outer >= 1, ell_inner_maxit >= 1 required");
  for (int k = 0; k < d->n_stim; ++k) {
    const ep_stim& s = d->stim[k];
    if (!std::isfinite(s.amp) || !std::isfinite(s.radius) || std::isnan(s.t_on) ||
        std::isnan(s.t_off))
      return fail(g, EP_ERR_ARG, "non-finite stimulus field");
  }

  std::copy(d->n, d->n + 3, g->n);
  g->arena = static_cast<char*>(d->arena);
  g->arena_bytes = d->arena ? d->arena_bytes : 0;
  g->h = d->h;
  g->dt = d->dt;
  g->model = d->model;
  g->prec = d->prec;
  g->diff = d->diff;
  g->ionic = d->ionic;
  g->theta = d->act_threshold;
  g->pcg_rtol = d->pcg_rtol;
  g->pcg_maxit = d->pcg_maxit;
  g->jacobi_sweeps = d->jacobi_sweeps;
  g->ell_rtol = d->ell_rtol;
  g->ell_max_outer = d->ell_max_outer;
  g->ell_inner_maxit = d->ell_inner_maxit;
  if (d->model == EP_BIDO && d->ell_precond != 0 && d->ell_precond != 1)
    return fail(g, EP_ERR_ARG, "ell_precond must be 0 (Jacobi + coarse) or 1 (Jacobi)");
  g->coarse_on = d->model == EP_BIDO && d->ell_precond == 0;
  g->stims.assign(d->stim, d->stim + d->n_stim);

  if (d->stream) {
    g->stream = static_cast<hipStream_t>(d->stream);
  } else {
    HIPCHK(g, hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    g->own_stream = true;
  }

  // brick map, over the heart and the bath
  const int64_t N = static_cast<int64_t>(g->n[0]) * g->n[1] * g->n[2];
  std::vector<uint8_t> boxmask(N, 1);
  if (d->mask)
    for (int64_t i = 0; i < N; ++i) boxmask[i] = d->mask[i] ? 1 : 0;
  g->bath = d->bath != nullptr;
  g->sig_bath = g->bath ? d->sig_bath : 0.0;
  if (g->bath) {
    for (int64_t i = 0; i < N; ++i) {
      if (!d->bath[i]) continue;
      if (boxmask[i]) return fail(g, EP_ERR_ARG, "bath voxels must lie outside the heart");
      boxmask[i] = 2;
    }
  }
  BrickMap bm;
  std::string merr;
  if (!build_brick_map(g->n, boxmask.data(), bm, merr)) return fail(g, EP_ERR_ARG, merr);
  g->nbx = bm.nbx;
  g->nby = bm.nby;
  g->nbz = bm.nbz;
  g->brick_id = std::move(bm.brick_id);
  g->brick_pos = std::move(bm.brick_pos);
  g->hbody = std::move(bm.mask);
  const int nb = bm.nb;
  g->nb = nb;
  g->n_body = bm.n_tissue;
  g->nvox = bm.nvox;
  // kernels address per-voxel arrays with 32-bit byte offsets, and some
  // arrays are FP64 (bidomain, FP64 state, the set-up's weight copy)
  if (g->nvox > (int64_t(1) << 29))
    return fail(g, EP_ERR_UNSUPPORTED, "grid too large: more than 2^29 voxels in active bricks");
  if (g->bath) {
    // the heart alone, in brick layout
    g->hmask.assign(g->hbody.size(), 0);
    g->n_tissue = 0;
    for (int x = 0; x < g->n[0]; ++x)
      for (int y = 0; y < g->n[1]; ++y)
        for (int z = 0; z < g->n[2]; ++z)
          if (boxmask[(static_cast<int64_t>(x) * g->n[1] + y) * g->n[2] + z] == 1) {
            g->hmask[brick_index(g, x, y, z)] = 1;
            ++g->n_tissue;
          }
  } else {
    g->hmask = g->hbody;
    g->n_tissue = g->n_body;
  }
  g->grid = grid_for(nb);
  g->L.nb = nb;
  g->L.grid = g->grid;
  g->L.pgrid = pgrid_for(nb, g->prec == EP_F64);
  g->L.stream_nt = static_cast<long long>(kBeArrays) * (nb + 1) * kBV *
                       (g->prec == EP_F64 ? 8 : 4) > kLlcBytes;
  g->L.stream = g->stream;
  // the elliptic inner solve's kernels need at most 74 VGPRs: three
  // 512-thread blocks fit per CU
  g->Le = g->L;
  g->Le.pgrid = std::min(g->grid, 3 * 256);
  if (d->steps_per_launch < 0) return fail(g, EP_ERR_ARG, "steps_per_launch must be >= 0");
  if (d->persistent_blocks != 0) {
    if (d->persistent_blocks < 0 || d->persistent_blocks % kXcd != 0)
      return fail(g, EP_ERR_ARG, "persistent_blocks must be 0 or a positive multiple of 8");
    g->L.pgrid = std::min(g->L.pgrid, static_cast<int>(d->persistent_blocks));
    g->Le.pgrid = std::min(g->Le.pgrid, static_cast<int>(d->persistent_blocks));
  }
  if (g->model == EP_BIDO && tissue_components(boxmask, g->n) != 1)
    return fail(g, EP_ERR_ARG, g->bath ? "heart and bath must be one face-connected component"
                                       : "bidomain tissue must be one face-connected component");
  const std::vector<int>& hnbr = bm.nbr;

  // device buffers
  const size_t es = elem_size(g->prec);
  const size_t vb = static_cast<size_t>(g->nvox) * es;
  TRY(dalloc(g, &g->d_nbr, hnbr.size() * sizeof(int)));
  TRY(dalloc(g, &g->d_rowsn, bm.rowsn.size() * sizeof(uint64_t)));
  g->L.rowsn = g->d_rowsn;
  g->Le.rowsn = g->d_rowsn;
  TRY(dalloc(g, &g->d_mask, static_cast<size_t>(g->nvox)));
  if (g->bath) TRY(dalloc(g, &g->d_body, static_cast<size_t>(g->nvox)));
  else g->d_body = g->d_mask;
  TRY(dalloc(g, &g->d_brick_id, g->brick_id.size() * sizeof(int)));
  for (int k = 0; k < 2; ++k) {
    TRY(dalloc(g, &g->d_v[k], vb));
    TRY(dalloc(g, &g->d_w[k], vb));
  }
  TRY(dalloc(g, &g->d_tact, vb));
  TRY(dalloc(g, &g->d_jstim, vb));
  for (int k = 0; k < 6; ++k) TRY(dalloc(g, &g->d_c[k], vb));
  TRY(dalloc(g, &g->d_partials, static_cast<size_t>(g->grid) * 4 * sizeof(double)));
  TRY(dalloc(g, &g->d_cg, 2 * sizeof(CGScalars)));
  for (int k = 0; k < 2; ++k)
    TRY(dalloc(g, &g->d_cgp[k], static_cast<size_t>(std::max(g->L.pgrid, g->Le.pgrid)) *
                                   kMaxPartials *
                                   sizeof(double)));
  TRY(dalloc(g, &g->d_flags, 4 * sizeof(int)));
  TRY(dalloc(g, &g->d_sums, 8 * sizeof(double)));
  TRY(dalloc(g, &g->d_qacc, sizeof(double)));
  TRY(dalloc(g, &g->d_qstep, sizeof(double)));
  TRY(dalloc(g, &g->d_phi, static_cast<size_t>(g->nvox) * sizeof(double)));
  if (g->diff == EP_DIFF_BE_PCG) {
    for (int k = 0; k < 2; ++k) {
      TRY(dalloc(g, &g->d_cr[k], vb));
      TRY(dalloc(g, &g->d_cs[k], vb));
      TRY(dalloc(g, &g->d_cw[k], vb));
    }
    for (int k = 0; k < 2; ++k) TRY(dalloc(g, &g->d_bprev[k], vb));
    for (int k = 0; k < kDRing; ++k) TRY(dalloc(g, &g->d_dprev[k], vb));
    for (int k = 0; k < 2; ++k) TRY(dalloc(g, &g->d_q[k], vb));
  }
  if (g->diff == EP_DIFF_BE_JACOBI) {
    TRY(dalloc(g, &g->d_dinv, vb));
    TRY(dalloc(g, &g->d_vs, vb));
    TRY(dalloc(g, &g->d_cr[0], vb));
  }
  if (g->model == EP_MONO && g->diff == EP_DIFF_EXPLICIT)
    for (int k = 0; k < 6; ++k) TRY(dalloc(g, &g->d_d0[k], vb));
  g->steps_per_launch = d->steps_per_launch;
  if (g->model == EP_MONO && g->diff == EP_DIFF_EXPLICIT && d->steps_per_launch != 1) {
    const int cap = g->prec == EP_F64 ? explicit_ms_capacity<double>()
                                      : explicit_ms_capacity<float>();
    if (nb <= std::min(cap, kMsMaxBricks)) {
      for (int k = 0; k < 2; ++k) TRY(dalloc(g, &g->d_xms[k], vb));
      TRY(dalloc(g, &g->d_bar, sizeof(unsigned)));
      g->ms_on = true;
    }
  }
  if (g->model == EP_BIDO) {
    const size_t b64 = static_cast<size_t>(g->nvox) * sizeof(double);
    const size_t b32 = static_cast<size_t>(g->nvox) * sizeof(float);
    TRY(dalloc(g, &g->d_vs, vb));
    for (int k = 0; k < 3; ++k) TRY(dalloc(g, &g->d_phi_hist[k], b64));
    TRY(dalloc(g, &g->d_r64, b64));
    for (int k = 0; k < 6; ++k) {
      TRY(dalloc(g, &g->d_ci64[k], b64));
      TRY(dalloc(g, &g->d_ck64[k], b64));
      TRY(dalloc(g, &g->d_ck32[k], b32));
    }
    TRY(dalloc(g, &g->d_x32, b32));
    for (int k = 0; k < 2; ++k) TRY(dalloc(g, &g->d_r32[k], b32));
    TRY(dalloc(g, &g->d_s32, b32));
    TRY(dalloc(g, &g->d_w32, b32));
    TRY(dalloc(g, &g->d_p32, b32));
    // aggregates: cubes of agg_edge^3 bricks, the smallest edge that keeps
    // their number within kMaxAgg; numbered in brick order
    for (g->agg_edge = 1;; g->agg_edge *= 2) {
      const int e = g->agg_edge;
      const int ax = (g->nbx + e - 1) / e, ay = (g->nby + e - 1) / e, az = (g->nbz + e - 1) / e;
      std::vector<int> id(static_cast<size_t>(ax) * ay * az, -1);
      std::vector<int> agg(nb + 1, 0);
      int na = 0;
      for (int b = 0; b < nb; ++b) {
        const int* bp = &g->brick_pos[3 * static_cast<size_t>(b)];
        int& a = id[(static_cast<size_t>(bp[0] / e) * ay + bp[1] / e) * az + bp[2] / e];
        if (a < 0) a = na++;
        agg[b] = a;
      }
      if (na > kMaxAgg) continue;
      agg[nb] = na;
      std::vector<int> ptr(na + 1, 0), brk(nb);
      for (int b = 0; b < nb; ++b) ++ptr[agg[b] + 1];
      for (int a = 0; a < na; ++a) ptr[a + 1] += ptr[a];
      std::vector<int> fill(ptr.begin(), ptr.end() - 1);
      for (int b = 0; b < nb; ++b) brk[fill[agg[b]]++] = b;
      g->n_agg = na;
      TRY(dalloc(g, &g->d_agg, agg.size() * sizeof(int)));
      TRY(dalloc(g, &g->d_agg_ptr, ptr.size() * sizeof(int)));
      TRY(dalloc(g, &g->d_agg_brk, brk.size() * sizeof(int)));
      HIPCHK(g, hipMemcpyAsync(g->d_agg, agg.data(), agg.size() * sizeof(int),
                               hipMemcpyHostToDevice, g->stream));
      HIPCHK(g, hipMemcpyAsync(g->d_agg_ptr, ptr.data(), ptr.size() * sizeof(int),
                               hipMemcpyHostToDevice, g->stream));
      HIPCHK(g, hipMemcpyAsync(g->d_agg_brk, brk.data(), brk.size() * sizeof(int),
                               hipMemcpyHostToDevice, g->stream));
      HIPCHK(g, hipStreamSynchronize(g->stream));
      break;
    }
    g->agg_ld = (g->n_agg + 3) & ~3;
    const size_t nrb = static_cast<size_t>(std::max(nb, g->agg_ld));
    TRY(dalloc(g, &g->d_rb, nrb * sizeof(float)));
    TRY(dalloc(g, &g->d_rc, static_cast<size_t>(g->agg_ld) * sizeof(float)));
    TRY(dalloc(g, &g->d_cc, static_cast<size_t>(g->n_agg + 1) * sizeof(float)));
    _Float16* kinv16 = nullptr;
    TRY(dalloc(g, &kinv16, static_cast<size_t>(g->n_agg) * g->agg_ld * sizeof(_Float16)));
    g->d_kinv = kinv16;
    HIPCHK(g, hipMemsetAsync(g->d_rb, 0, nrb * sizeof(float), g->stream));
    HIPCHK(g, hipMemsetAsync(g->d_rc, 0, static_cast<size_t>(g->agg_ld) * sizeof(float),
                             g->stream));
    HIPCHK(g, hipMemsetAsync(g->d_cc, 0, static_cast<size_t>(g->n_agg + 1) * sizeof(float),
                             g->stream));
    TRY(dalloc(g, &g->d_dinvk, b32));
  }
  {
    void* p = nullptr;
    HIPCHK(g, hipHostMalloc(&p, sizeof(HostSync), hipHostMallocDefault));
    g->hs = static_cast<HostSync*>(p);
    std::memset(g->hs, 0, sizeof(HostSync));
    void* m = nullptr;
    HIPCHK(g, hipHostMalloc(&m, 64, hipHostMallocMapped | hipHostMallocCoherent));
    g->hmirror = static_cast<volatile unsigned long long*>(m);
    *g->hmirror = 0;
    void* dm = nullptr;
    HIPCHK(g, hipHostGetDevicePointer(&dm, m, 0));
    g->dmirror = static_cast<unsigned long long*>(dm);
  }
  HIPCHK(g, hipMemcpyAsync(g->d_nbr, hnbr.data(), hnbr.size() * sizeof(int),
                           hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipMemcpyAsync(g->d_rowsn, bm.rowsn.data(), bm.rowsn.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipMemcpyAsync(g->d_brick_id, g->brick_id.data(), g->brick_id.size() * sizeof(int),
                           hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipMemcpyAsync(g->d_mask, g->hmask.data(), g->hmask.size(), hipMemcpyHostToDevice,
                           g->stream));
  if (g->bath)
    HIPCHK(g, hipMemcpyAsync(g->d_body, g->hbody.data(), g->hbody.size(), hipMemcpyHostToDevice,
                             g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  TRY(build_stimuli(g));
  // initial state: v = 0, w = 1 (tissue and non-tissue of active bricks), T_act = +inf
  std::vector<double> zero(N, 0.0), inf(N, kInf);
  TRY(ep_write_state(g, EP_V, zero.data(), N));
  {
    std::vector<double> one(N, 1.0);
    TRY(ep_write_state(g, EP_W, one.data(), N));
  }
  TRY(ep_write_state(g, EP_TACT, inf.data(), N));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return EP_OK;
}

template <typename T>
ep_status write_field(ep_grid g, ep_field f, const double* in) {
  const size_t es = (f == EP_PHIE) ? sizeof(double) : sizeof(T);
  std::vector<unsigned char> buf(static_cast<size_t>(g->nvox) * es, 0);
  T* bt = reinterpret_cast<T*>(buf.data());
  double* bd = reinterpret_cast<double*>(buf.data());
  const int64_t nreal = static_cast<int64_t>(g->nb) * kBV;
  // defaults for non-tissue voxels of active bricks (the ghost brick stays 0)
  if (f == EP_W || f == EP_TACT) {
    const T fill = f == EP_W ? T(1) : static_cast<T>(kInf);
    std::fill(bt, bt + nreal, fill);
  }
  parallel_for(g->n[0], [&](int64_t x) {
    for (int y = 0; y < g->n[1]; ++y)
      for (int z = 0; z < g->n[2]; ++z) {
        const int64_t gi = brick_index(g, static_cast<int>(x), y, z);
        const std::vector<uint8_t>& m = (f == EP_PHIE) ? g->hbody : g->hmask;
        if (gi < 0 || !m[gi]) continue;
        const double v = in[box_index(g, static_cast<int>(x), y, z)];
        if (f == EP_PHIE) bd[gi] = v;
        else bt[gi] = static_cast<T>(v);
      }
  });
  void* dst = nullptr;
  switch (f) {
    case EP_V: dst = g->d_v[g->cur]; break;
    case EP_W: dst = g->d_w[g->cur]; break;
    case EP_PHIE: dst = g->d_phi; break;
    case EP_TACT: dst = g->d_tact; break;
  }
  HIPCHK(g, hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return EP_OK;
}

template <typename T>
ep_status read_field(ep_grid g, ep_field f, double* out) {
  const size_t es = (f == EP_PHIE) ? sizeof(double) : sizeof(T);
  std::vector<unsigned char> buf(static_cast<size_t>(g->nvox) * es);
  const void* src = nullptr;
  switch (f) {
    case EP_V: src = g->d_v[g->cur]; break;
    case EP_W: src = g->d_w[g->cur]; break;
    case EP_PHIE: src = g->d_phi; break;
    case EP_TACT: src = g->d_tact; break;
  }
  HIPCHK(g, hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  const T* bt = reinterpret_cast<const T*>(buf.data());
  const double* bd = reinterpret_cast<const double*>(buf.data());
  const double off = (f == EP_TACT) ? kInf : 0.0;
  parallel_for(g->n[0], [&](int64_t x) {
    for (int y = 0; y < g->n[1]; ++y)
      for (int z = 0; z < g->n[2]; ++z) {
        const int64_t gi = brick_index(g, static_cast<int>(x), y, z);
        double v = off;
        const std::vector<uint8_t>& m = (f == EP_PHIE) ? g->hbody : g->hmask;
        if (gi >= 0 && m[gi]) v = (f == EP_PHIE) ? bd[gi] : static_cast<double>(bt[gi]);
        out[box_index(g, static_cast<int>(x), y, z)] = v;
      }
  });
  return EP_OK;
}

ep_status set_cond_impl(ep_grid g, const double* fibre, const double* scale, double sl,
                        double st, double sel, double set_) {
  if (!fibre) return fail(g, EP_ERR_ARG, "fibre is NULL");
  if (!(sl >= 0) || !(st >= 0) || !std::isfinite(sl) || !std::isfinite(st))
    return fail(g, EP_ERR_ARG, "conductivities must be finite and >= 0");
  if (g->model == EP_BIDO && (!(sel >= 0) || !(set_ >= 0) || !std::isfinite(sel) ||
                              !std::isfinite(set_)))
    return fail(g, EP_ERR_ARG, "extracellular conductivities must be finite and >= 0");
  // fibres / scale to brick layout, validated on tissue
  std::vector<double> hf(static_cast<size_t>(g->nvox) * 3, 0.0), hsc;
  if (scale) hsc.assign(g->nvox, 0.0);
  std::atomic<int> bad{0};   // 1: non-unit fibre, 2: bad scale
  parallel_for(g->n[0], [&](int64_t xx) {
    const int x = static_cast<int>(xx);
    for (int y = 0; y < g->n[1]; ++y)
      for (int z = 0; z < g->n[2]; ++z) {
        const int64_t gi = brick_index(g, x, y, z);
        if (gi < 0 || !g->hmask[gi]) continue;
        const int64_t bi = box_index(g, x, y, z);
        const double f0 = fibre[3 * bi], f1 = fibre[3 * bi + 1], f2 = fibre[3 * bi + 2];
        const double nrm = std::sqrt(f0 * f0 + f1 * f1 + f2 * f2);
        if (!(std::fabs(nrm - 1.0) <= 1e-6)) bad.store(1);
        hf[3 * gi] = f0;
        hf[3 * gi + 1] = f1;
        hf[3 * gi + 2] = f2;
        if (scale) {
          const double s = scale[bi];
          if (!(s > 0) || !std::isfinite(s)) bad.store(2);
          hsc[gi] = s;
        }
      }
  });
  if (bad.load() == 1) return fail(g, EP_ERR_ARG, "fibre is not a unit vector on a tissue voxel");
  if (bad.load() == 2) return fail(g, EP_ERR_ARG, "scale must be finite and > 0 on tissue");
  double *dfib = nullptr, *dsc = nullptr, *tens = nullptr;
  const size_t b64 = static_cast<size_t>(g->nvox) * sizeof(double);
  Temps tmp(g);
  hipError_t e = tmp.get(&dfib, 3 * b64);
  if (e == hipSuccess && scale) e = tmp.get(&dsc, b64);
  if (e == hipSuccess) e = tmp.get(&tens, 6 * b64);
  double* tmp64[6] = {};
  const bool need64 = (g->prec == EP_F64) || g->model == EP_BIDO || g->diff == EP_DIFF_EXPLICIT;
  if (e == hipSuccess && need64)
    for (int k = 0; k < 6 && e == hipSuccess; ++k) e = tmp.get(&tmp64[k], b64);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(g, EP_ERR_OOM, g->arena ? "arena too small for the coefficient-encoding "
                                          "temporaries (ep_grid_stats reports the peak)"
                                        : "temporary allocation for coefficient encoding failed");
  }
  ep_status rc = EP_OK;
  do {
    if (hipMemcpyAsync(dfib, hf.data(), 3 * b64, hipMemcpyHostToDevice, g->stream) != hipSuccess ||
        (scale && hipMemcpyAsync(dsc, hsc.data(), b64, hipMemcpyHostToDevice, g->stream) != hipSuccess) ||
        hipMemsetAsync(tens, 0, 6 * b64, g->stream) != hipSuccess) {
      rc = fail(g, EP_ERR_HIP, "upload of fibres failed");
      break;
    }
    // the ghost brick of every coefficient array must read zero
    for (int k = 0; k < 6 && tmp64[k]; ++k)
      if (hipMemsetAsync(tmp64[k], 0, b64, g->stream) != hipSuccess) rc = EP_ERR_HIP;
    if (rc != EP_OK) {
      rc = fail(g, EP_ERR_HIP, "clearing coefficient scratch failed");
      break;
    }
    // monodomain / intracellular set in state precision (+ FP64 twin for checks)
    float* c32[6];
    double* c64[6];
    for (int k = 0; k < 6; ++k) {
      c32[k] = static_cast<float*>(g->d_c[k]);
      c64[k] = g->model == EP_BIDO ? g->d_ci64[k] : tmp64[k];
    }
    if (g->prec == EP_F64)
      for (int k = 0; k < 6; ++k) c64[k] = static_cast<double*>(g->d_c[k]);
    if (g->diff == EP_DIFF_EXPLICIT27)
      launch_corner_coefs(g->L, g->d_nbr, g->d_mask, dfib, dsc, sl, st, g->h, tens,
                          need64 ? c64 : nullptr, g->prec == EP_F32 ? c32 : nullptr);
    else
      launch_tensor_coefs(g->L, g->d_nbr, g->d_mask, dfib, dsc, sl, st, g->h, tens,
                          need64 ? c64 : nullptr, g->prec == EP_F32 ? c32 : nullptr);
    if (g->model == EP_MONO && g->diff == EP_DIFF_EXPLICIT) {
      if (g->prec == EP_F64)
        launch_unit_tensors<double>(g->L, g->d_mask, dfib, sl, st,
                                    reinterpret_cast<double**>(g->d_d0));
      else
        launch_unit_tensors<float>(g->L, g->d_mask, dfib, sl, st,
                                   reinterpret_cast<float**>(g->d_d0));
    }
    if (g->model == EP_BIDO) {
      if (g->prec == EP_F64) {
        // FP64 state: d_c already holds A_i in FP64; copy it into the FP64 twin
        for (int k = 0; k < 6; ++k)
          (void)hipMemcpyAsync(g->d_ci64[k], g->d_c[k], b64, hipMemcpyDeviceToDevice, g->stream);
      }
      // K = -(A_i + A_e), each part over its own domain (eqn:bidomain1 and
      // its boundary conditions): A_i with the intracellular tensor on the
      // heart only (no intracellular current crosses the heart's boundary),
      // A_e over the elliptic domain with D_e on the heart and, with a bath,
      // sig_bath I on the bath (faces straddling the two take the mean).
      // The weights of a sum of operators are the sums of their weights.
      launch_tensor_coefs(g->L, g->d_nbr, g->d_mask, dfib, dsc, sel, set_, g->h, tens,
                          g->d_ck64, nullptr, g->bath ? g->d_body : nullptr, g->sig_bath);
      launch_coef_add(g->L, g->d_ck64, g->d_ci64, g->d_ck32);
      launch_dinv<float>(g->L, g->d_nbr, cset32(g->d_ck32), 0.0f, -1.0f, g->d_dinvk);
      if (g->coarse_on) {
        rc = coarse_setup(g, tmp);
        if (rc != EP_OK) break;
      }
    }
    if (g->diff == EP_DIFF_BE_JACOBI) {
      if (g->prec == EP_F64)
        launch_dinv<double>(g->L, g->d_nbr, coefs<double>(g), 1.0, -g->dt,
                            static_cast<double*>(g->d_dinv));
      else
        launch_dinv<float>(g->L, g->d_nbr, coefs<float>(g), 1.0f, static_cast<float>(-g->dt),
                           static_cast<float*>(g->d_dinv));
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(g->stream) != hipSuccess) {
      rc = fail(g, EP_ERR_HIP, "coefficient kernels failed");
      break;
    }
    if (g->diff == EP_DIFF_EXPLICIT) {
      double* const* cc = (g->prec == EP_F64) ? reinterpret_cast<double* const*>(g->d_c)
                                              : (g->model == EP_BIDO ? g->d_ci64 : tmp64);
      rc = check_explicit_stability(g, cc);
    } else if (g->diff == EP_DIFF_EXPLICIT27) {
      // lambda_max(-A27) <= 4 max_p lambda_max(D_p) / h^2: each of a voxel's 8
      // corners adds a term of norm lambda_max(D_c) / (2 h^2), and D_c is a mean
      // of voxel tensors whose largest eigenvalue is s_p max(sL, sT) (unit
      // fibres, to the 1e-6 checked above).  Uniform tissue comes within a
      // few per cent of it, so the bound is the test.
      double smax = 1.0;
      if (scale) {
        smax = 0.0;
        for (int64_t i = 0; i < g->nvox; ++i)
          if (g->hmask[i]) smax = std::max(smax, hsc[i]);
      }
      const double lam = 4.0 * smax * std::max(sl, st) * (1.0 + 1e-5) / (g->h * g->h);
      if (!(g->dt * lam < 2.0)) {
        char buf[160];
        snprintf(buf, sizeof buf, "explicit diffusion unstable: dt*lambda_max(-A27) <= %.3f "
                 "is not below 2", g->dt * lam);
        rc = fail(g, EP_ERR_ARG, buf);
      }
    }
  } while (false);
  (void)hipStreamSynchronize(g->stream);
  if (rc == EP_OK) g->has_cond = true;
  g->have_bprev = false;
  g->pred_len = 0;
  return rc;
}

// Bytes of device temporaries set_cond_impl takes for grid g (each
// request rounded to 256 bytes, as Temps carves them): fibres, scale, voxel
// tensors, the FP64 weight scratch, the power-iteration vectors of the
// explicit stability estimate, and the coarse operator's set-up.
size_t cond_temp_bytes(const ep_grid g, bool has_scale) {
  auto al = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
  const size_t b64 = static_cast<size_t>(g->nvox) * sizeof(double);
  const bool need64 = (g->prec == EP_F64) || g->model == EP_BIDO || g->diff == EP_DIFF_EXPLICIT;
  size_t need = al(3 * b64) + (has_scale ? al(b64) : 0) + al(6 * b64);
  if (need64) need += 6 * al(b64);
  if (g->diff == EP_DIFF_EXPLICIT) need += 2 * al(b64);
  if (g->model == EP_BIDO && g->coarse_on) {
    const size_t n = static_cast<size_t>(g->n_agg);
    need += al(static_cast<size_t>(g->nb) * kCoarseRow * sizeof(double)) +
            al(n * n * sizeof(double)) + al(kGjPanel * kGjPanel * sizeof(double)) +
            2 * al(kGjPanel * n * sizeof(double));
  }
  return need;
}

}  // namespace

// Scratch of the allocation-free conductivity set-up: one copy per GPU the
// library runs on, held until the process ends.  Host code never passes its
// name to a kernel or a copy (on the host it is only a stand-in for the
// symbol); it uses the device address looked up once per device below.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (hipGetSymbolAddress with the
// device current, once per device).
ep_status scratch_on(ep_grid g, void** out) {
  if (g->device < 0 || g->device >= kMaxDevices)
    return fail(g, EP_ERR_UNSUPPORTED, "device id beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[g->device]) {
    int prev = 0;
    HIPCHK(g, hipGetDevice(&prev));
    if (prev != g->device) HIPCHK(g, hipSetDevice(g->device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != g->device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p)
      return fail(g, EP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[g->device] = p;
  }
  *out = g_scratch_ptr[g->device];
  return EP_OK;
}

}  // namespace

extern "C" {

EP_API ep_status ep_create_grid(const ep_grid_desc* d, ep_grid* out) {
  if (!out) return EP_ERR_ARG;
  *out = nullptr;
  if (!d) return EP_ERR_ARG;
  ep_grid g = new (std::nothrow) ep_grid_s();
  if (!g) return EP_ERR_OOM;
  ep_status s;
  try {
    s = create_impl(d, g);
  } catch (const std::bad_alloc&) {
    s = fail(g, EP_ERR_OOM, "host allocation failed");
  } catch (...) {
    s = fail(g, EP_ERR_HIP, "unexpected exception");
  }
  if (s != EP_OK) {
    create_error() = g->err;
    ep_destroy_grid(g);
    return s;
  }
  *out = g;
  return EP_OK;
}

EP_API ep_status ep_set_conductivity_fibres(ep_grid g, const double* fibre, const double* scale,
                                            double sig_l, double sig_t, double sig_el,
                                            double sig_et) {
  if (!g) return EP_ERR_ARG;
  try {
    return set_cond_impl(g, fibre, scale, sig_l, sig_t, sig_el, sig_et);
  } catch (const std::bad_alloc&) {
    return fail(g, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_set_conductivity_fibres_noalloc(ep_grid g, const double* fibre,
                                                    const double* scale, double sig_l,
                                                    double sig_t, double sig_el,
                                                    double sig_et) {
  if (!g) return EP_ERR_ARG;
  const size_t need = cond_temp_bytes(g, scale != nullptr);
  if (need > kNoAllocScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf, "the conductivity set-up of this grid needs %zu bytes of "
             "device temporaries; the allocation-free call holds at most %zu", need,
             kNoAllocScratchBytes);
    return fail(g, EP_ERR_ARG, buf);
  }
  void* base = nullptr;
  TRY(scratch_on(g, &base));
  g->temp_region = static_cast<char*>(base);
  g->temp_cap = kNoAllocScratchBytes;
  g->temp_used = 0;
  ep_status rc;
  try {
    rc = set_cond_impl(g, fibre, scale, sig_l, sig_t, sig_el, sig_et);
  } catch (const std::bad_alloc&) {
    rc = fail(g, EP_ERR_OOM, "host allocation failed");
  }
  g->temp_region = nullptr;
  g->temp_cap = 0;
  g->temp_used = 0;
  return rc;
}

EP_API ep_status ep_step(ep_grid g, int32_t nsteps, ep_step_info* info) {
  if (!g) return EP_ERR_ARG;
  if (nsteps < 0) return fail(g, EP_ERR_ARG, "nsteps must be >= 0");
  if (!g->has_cond) return fail(g, EP_ERR_STATE, "ep_set_conductivity_fibres not called");
  if (g->nonfinite) return fail(g, EP_ERR_NONFINITE, "state is non-finite; write a new state");
  try {
    return g->prec == EP_F64 ? run_steps<double>(g, nsteps, info)
                             : run_steps<float>(g, nsteps, info);
  } catch (const std::bad_alloc&) {
    return fail(g, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_adjoint_scale(ep_grid g, int32_t nsteps, int32_t ckpt_every,
                                  const double* tstar, double* loss, double* grad,
                                  int64_t* n_used) {
  if (!g) return EP_ERR_ARG;
  if (!tstar || !loss || !n_used) return fail(g, EP_ERR_ARG, "NULL argument");
  if (nsteps < 1) return fail(g, EP_ERR_ARG, "nsteps must be >= 1");
  if (ckpt_every < 0) return fail(g, EP_ERR_ARG, "ckpt_every must be >= 0");
  if (g->model != EP_MONO || g->diff != EP_DIFF_EXPLICIT)
    return fail(g, EP_ERR_UNSUPPORTED, "the adjoint covers the explicit monodomain step only");
  if (!g->has_cond) return fail(g, EP_ERR_STATE, "ep_set_conductivity_fibres not called");
  if (g->nonfinite) return fail(g, EP_ERR_NONFINITE, "state is non-finite; write a new state");
  int32_t K = ckpt_every;
  if (K == 0) K = std::max(1, static_cast<int32_t>(std::lround(std::sqrt(1.5 * nsteps))));
  K = std::min(K, nsteps);
  try {
    return g->prec == EP_F64 ? adjoint_impl<double>(g, nsteps, K, tstar, loss, grad, n_used)
                             : adjoint_impl<float>(g, nsteps, K, tstar, loss, grad, n_used);
  } catch (const std::bad_alloc&) {
    return fail(g, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_solve_elliptic(ep_grid g, double rel_tol, int32_t max_outer,
                                   ep_solve_info* info) {
  if (!g) return EP_ERR_ARG;
  if (g->model != EP_BIDO) return fail(g, EP_ERR_UNSUPPORTED, "monodomain grid");
  if (!g->has_cond) return fail(g, EP_ERR_STATE, "ep_set_conductivity_fibres not called");
  if (!(rel_tol > 0) || max_outer < 1) return fail(g, EP_ERR_ARG, "rel_tol > 0, max_outer >= 1");
  g->phi_hist = 0;   // this phi belongs to no step
  ep_status s = g->prec == EP_F64
                    ? elliptic<double>(g, static_cast<const double*>(g->d_v[g->cur]), rel_tol,
                                       max_outer, info)
                    : elliptic<float>(g, static_cast<const float*>(g->d_v[g->cur]), rel_tol,
                                      max_outer, info);
  if (hipStreamSynchronize(g->stream) != hipSuccess)
    return fail(g, EP_ERR_HIP, "stream synchronisation failed");
  if (s == EP_ERR_NOCONV) return fail(g, s, "elliptic refinement did not converge");
  return s;
}

EP_API ep_status ep_read_state(ep_grid g, ep_field f, double* host_out, size_t n) {
  if (!g || !host_out) return EP_ERR_ARG;
  if (f < EP_V || f > EP_TACT) return fail(g, EP_ERR_ARG, "bad field");
  const size_t N = static_cast<size_t>(g->n[0]) * g->n[1] * g->n[2];
  if (n < N) return fail(g, EP_ERR_ARG, "output buffer too small");
  try {
    return g->prec == EP_F64 ? read_field<double>(g, f, host_out) : read_field<float>(g, f, host_out);
  } catch (const std::bad_alloc&) {
    return fail(g, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_read_state_device(ep_grid g, ep_field f, void* dptr, int32_t dtype) {
  if (!g || !dptr) return EP_ERR_ARG;
  if (f < EP_V || f > EP_TACT) return fail(g, EP_ERR_ARG, "bad field");
  if (dtype != 0 && dtype != 1) return fail(g, EP_ERR_ARG, "dtype must be 0 (FP64) or 1 (FP32)");
  const void* src = nullptr;
  switch (f) {
    case EP_V: src = g->d_v[g->cur]; break;
    case EP_W: src = g->d_w[g->cur]; break;
    case EP_PHIE: src = g->d_phi; break;
    case EP_TACT: src = g->d_tact; break;
  }
  const double fill = (f == EP_TACT) ? kInf : 0.0;
  const uint8_t* fm = (f == EP_PHIE) ? g->d_body : g->d_mask;
  const bool src64 = (f == EP_PHIE) || g->prec == EP_F64;
  if (src64 && dtype == 0)
    launch_box_gather<double, double>(g->stream, g->n, g->nby, g->nbz, g->d_brick_id,
                                      static_cast<const double*>(src), fm,
                                      static_cast<double*>(dptr), fill);
  else if (src64)
    launch_box_gather<double, float>(g->stream, g->n, g->nby, g->nbz, g->d_brick_id,
                                     static_cast<const double*>(src), fm,
                                     static_cast<float*>(dptr), static_cast<float>(fill));
  else if (dtype == 0)
    launch_box_gather<float, double>(g->stream, g->n, g->nby, g->nbz, g->d_brick_id,
                                     static_cast<const float*>(src), fm,
                                     static_cast<double*>(dptr), fill);
  else
    launch_box_gather<float, float>(g->stream, g->n, g->nby, g->nbz, g->d_brick_id,
                                    static_cast<const float*>(src), fm,
                                    static_cast<float*>(dptr), static_cast<float>(fill));
  HIPCHK(g, hipGetLastError());
  return EP_OK;
}

EP_API ep_status ep_ecg_leads(ep_grid g, const int32_t* electrodes, double* out) {
  if (!g || !electrodes || !out) return EP_ERR_ARG;
  if (g->model != EP_BIDO)
    return fail(g, EP_ERR_UNSUPPORTED, "ECG leads need the bidomain extracellular potential");
  int64_t gi[3];
  for (int k = 0; k < 3; ++k) {
    const int x = electrodes[3 * k], y = electrodes[3 * k + 1], z = electrodes[3 * k + 2];
    if (x < 0 || y < 0 || z < 0 || x >= g->n[0] || y >= g->n[1] || z >= g->n[2])
      return fail(g, EP_ERR_ARG, "electrode outside the box");
    gi[k] = brick_index(g, x, y, z);
    if (gi[k] < 0 || !g->hbody[gi[k]])
      return fail(g, EP_ERR_ARG, "electrode outside the elliptic domain (heart or bath)");
  }
  for (int k = 0; k < 3; ++k)
    HIPCHK(g, hipMemcpyAsync(&g->hs->sums[k], g->d_phi + gi[k], sizeof(double),
                             hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  const double ra = g->hs->sums[0], la = g->hs->sums[1], ll = g->hs->sums[2];
  out[0] = la - ra;
  out[1] = ll - ra;
  out[2] = ll - la;
  out[3] = ra - 0.5 * (la + ll);
  out[4] = la - 0.5 * (ra + ll);
  out[5] = ll - 0.5 * (ra + la);
  return EP_OK;
}

EP_API ep_status ep_write_state(ep_grid g, ep_field f, const double* host_in, size_t n) {
  if (!g || !host_in) return EP_ERR_ARG;
  if (f < EP_V || f > EP_TACT) return fail(g, EP_ERR_ARG, "bad field");
  const size_t N = static_cast<size_t>(g->n[0]) * g->n[1] * g->n[2];
  if (n < N) return fail(g, EP_ERR_ARG, "input buffer too small");
  try {
    ep_status s = g->prec == EP_F64 ? write_field<double>(g, f, host_in)
                                    : write_field<float>(g, f, host_in);
    if (s == EP_OK) {
      if (f == EP_V) g->have_prev = false;
      g->have_bprev = false;
      g->pred_len = 0;
      g->phi_hist = 0;
      g->nonfinite = false;
      HIPCHK(g, hipMemsetAsync(g->d_flags, 0, 4 * sizeof(int), g->stream));
      HIPCHK(g, hipStreamSynchronize(g->stream));
    }
    return s;
  } catch (const std::bad_alloc&) {
    return fail(g, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_get_step(ep_grid g, int64_t* step) {
  if (!g || !step) return EP_ERR_ARG;
  *step = g->step;
  return EP_OK;
}

EP_API ep_status ep_set_step(ep_grid g, int64_t step) {
  if (!g || step < 0) return EP_ERR_ARG;
  g->step = step;
  g->stim_built = false;
  g->have_prev = false;
  g->have_bprev = false;
  g->pred_len = 0;
  g->phi_hist = 0;
  return EP_OK;
}

EP_API ep_status ep_grid_stats(ep_grid g, int64_t* n_tissue, int64_t* n_bricks,
                               int64_t* device_bytes) {
  if (!g) return EP_ERR_ARG;
  if (n_tissue) *n_tissue = g->n_tissue;
  if (n_bricks) *n_bricks = g->nb;
  if (device_bytes) *device_bytes = g->dev_peak;
  return EP_OK;
}

EP_API ep_status ep_kernel_timing(ep_grid g, int32_t enable) {
  if (!g) return EP_ERR_ARG;
  g->timing = static_cast<uint32_t>(enable) & ((1u << kTimers) - 1u);
  for (int k = 0; k < kTimers; ++k) {
    g->tms[k] = 0;
    g->tcount[k] = 0;
    g->tused[k] = 0;
  }
  return EP_OK;
}

EP_API ep_status ep_kernel_timing_period(ep_grid g, int32_t steps) {
  if (!g || steps < 1) return EP_ERR_ARG;
  g->timing_period = steps;
  return EP_OK;
}

EP_API ep_status ep_kernel_time(ep_grid g, int32_t kernel_id, double* total_ms,
                                int64_t* launches) {
  if (!g || kernel_id < 0 || kernel_id >= kTimers) return EP_ERR_ARG;
  if (total_ms) *total_ms = g->tms[kernel_id];
  if (launches) *launches = g->tcount[kernel_id];
  return EP_OK;
}

EP_API ep_status ep_destroy_grid(ep_grid g) {
  if (!g) return EP_ERR_ARG;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (void* p : g->allocs) (void)hipFree(p);
  if (g->d_adj && !g->adj_in_arena) (void)hipFree(g->d_adj);
  for (int k = 0; k < kTimers; ++k)
    for (auto& tp : g->tk[k]) {
      (void)hipEventDestroy(tp.a);
      (void)hipEventDestroy(tp.b);
    }
  if (g->hs) (void)hipHostFree(g->hs);
  if (g->hmirror) (void)hipHostFree(const_cast<unsigned long long*>(g->hmirror));
  if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
  return EP_OK;
}

EP_API const char* ep_status_string(ep_status s) {
  switch (s) {
    case EP_OK: return "EP_OK";
    case EP_ERR_ARG: return "EP_ERR_ARG";
    case EP_ERR_OOM: return "EP_ERR_OOM";
    case EP_ERR_HIP: return "EP_ERR_HIP";
    case EP_ERR_NOCONV: return "EP_ERR_NOCONV";
    case EP_ERR_NONFINITE: return "EP_ERR_NONFINITE";
    case EP_ERR_STATE: return "EP_ERR_STATE";
    case EP_ERR_UNSUPPORTED: return "EP_ERR_UNSUPPORTED";
  }
  return "EP_ERR_UNKNOWN";
}

EP_API const char* ep_last_error(ep_grid g) {
  return g ? g->err.c_str() : create_error().c_str();
}

}  // extern "C"

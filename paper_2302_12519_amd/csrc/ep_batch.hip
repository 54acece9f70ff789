// Batched serving of many explicit-monodomain simulations on one GPU (the
// ep_batch_* family of include/ep.h).
//
// Device side: every admitted request ("slot") owns a region of one arena
// allocation holding its neighbour table, FP32 operator weights, ping-pong
// v / w, activation times and stimulus amplitudes.  A work list of
// (slot, brick) pairs lists every brick of every running request; one
// persistent launch of k_batch_step (a fixed grid of resident blocks that
// strides over the list) advances all of them by one step, each
// brick with exactly the per-grid explicit kernel's arithmetic (so a request
// gives the same bits alone, in any mix, or through ep_step).  The state of
// step s lives in buffer s & 1, and a launch for substep k skips slots whose
// step + k has reached their own step count.  K substeps plus a counter
// update are captured once in a hipGraph; admission and retirement only
// rewrite the slot table and the work list between graph launches.  A new
// request's region is built on a stream of its own while the graph launch
// in flight runs; the next launch waits for it.
//
// Host side: FIFO admission by HBM budget (first-fit arena with coalescing)
// and free slots, request bookkeeping and result read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "ep_device.h"
#include "ep_layout.h"

namespace ep {
namespace {

using namespace dev;

struct SlotDev {
  const int* nbr;
  const uint64_t* rowsn;  // (nb + 1) * 27 row masks of each brick's neighbourhood
  const float* c[6];
  float* v[2];
  float* w[2];
  float* tact;
  const float* jamp;      // stimulus current per voxel while the window is open
  IonicT<float> ion;
  float dt, theta;
  double dtd, t_on, t_off;
  long long step, n_steps;
  int active, nb;         // nb: active bricks (the ghost brick's id)
};

struct WorkItem {
  int slot, brick;
};

// A slot's buffers are device memory, but pointers read from memory are
// generic to the compiler: its accesses through them would be flat ones,
// which take a 64-bit address per lane and count against the LDS counter
// too (so every LDS wait would also wait for memory).  These load and store
// element i through the global address space, as a scalar base plus a
// 32-bit byte offset, like at().
template <typename T>
__device__ __forceinline__ T gld(const T* p, int i) {
  using GC = __attribute__((address_space(1))) const char*;
  using GT = __attribute__((address_space(1))) const T*;
  return *(GT)((GC)p + static_cast<uint64_t>(static_cast<uint32_t>(i) *
                                             static_cast<uint32_t>(sizeof(T))));
}
template <typename T>
__device__ __forceinline__ void gst(T* p, int i, T v) {
  using GC = __attribute__((address_space(1))) char*;
  using GT = __attribute__((address_space(1))) T*;
  *(GT)((GC)p + static_cast<uint64_t>(static_cast<uint32_t>(i) *
                                      static_cast<uint32_t>(sizeof(T)))) = v;
}
struct GLoad {
  template <typename T>
  __device__ __forceinline__ T operator()(const T* p, int i) const { return gld(p, i); }
};

// One explicit step of every running request's bricks (substep k of the
// current graph launch).  Persistent: the work list is dealt to the 8 XCDs
// in contiguous ranges (a request's bricks are consecutive in the list, so
// halo neighbours tend to share an XCD's L2), and each block strides
// through its XCD's range.  The work record and neighbour row of a block's
// next brick are loaded one brick ahead, so the dependent metadata chain
// (work item -> slot -> neighbour row) overlaps the current brick.  Each
// brick takes exactly the per-grid explicit kernel's arithmetic.
__global__ __launch_bounds__(kBV) __attribute__((amdgpu_waves_per_eu(6))) void k_batch_step(const SlotDev* __restrict__ slots,
                                                    const WorkItem* __restrict__ work,
                                                    const int* __restrict__ count, int k,
                                                    int* flags) {
  __shared__ float s[kTile];
  __shared__ int nbs[2][kNbr];
  __shared__ uint64_t rows[2][kNbr];
  const int n = *count;
  const int xcd = blockIdx.x % kXcd, gper = gridDim.x / kXcd;
  const int per = (n + kXcd - 1) / kXcd;
  const int hi = min(n, (xcd + 1) * per);
  int i = xcd * per + static_cast<int>(blockIdx.x) / kXcd;
  WorkItem it{0, 0};
  int nbv = 0;
  uint64_t rmv = 0;
  if (i < hi) {
    it = work[i];
    if (threadIdx.x < kNbr) {
      nbv = gld(slots[it.slot].nbr, it.brick * kNbr + threadIdx.x);
      rmv = gld(slots[it.slot].rowsn, it.brick * kNbr + threadIdx.x);
    }
  }
  int buf = 0;
  for (; i < hi; i += gper) {
    if (threadIdx.x < kNbr) {
      nbs[buf][threadIdx.x] = nbv;
      rows[buf][threadIdx.x] = rmv;
    }
    // publishes this brick's neighbour row and row masks; every thread has
    // also finished reading the previous brick's tile
    __syncthreads();
    const SlotDev* sd = slots + it.slot;
    const int brick = it.brick;
    // the next brick's work record, neighbour row and row masks
    const int i2 = i + gper;
    WorkItem it2{0, 0};
    int nbv2 = 0;
    uint64_t rmv2 = 0;
    if (i2 < hi) {
      it2 = work[i2];
      if (threadIdx.x < kNbr) {
        nbv2 = gld(slots[it2.slot].nbr, it2.brick * kNbr + threadIdx.x);
        rmv2 = gld(slots[it2.slot].rowsn, it2.brick * kNbr + threadIdx.x);
      }
    }
    const long long st = sd->step + k;
    if (st < sd->n_steps) {
      const int* nb = nbs[buf];
      const uint64_t* rowm = rows[buf];
      const int ghost = sd->nb;
      const int par = static_cast<int>(st & 1);
      const float* __restrict__ v = sd->v[par];
      const float* __restrict__ w = sd->w[par];
      float* __restrict__ vout = sd->v[par ^ 1];
      float* __restrict__ wout = sd->w[par ^ 1];
      float* __restrict__ tact = sd->tact;
      const double tn = static_cast<double>(st) * sd->dtd;
      const float* __restrict__ jstim =
          (sd->jamp && sd->t_on <= tn && tn < sd->t_off) ? sd->jamp : nullptr;
      const IonicT<float> ion = sd->ion;
      const float dt = sd->dt, theta = sd->theta;
      CoefSet<float> c;
      for (int q = 0; q < 6; ++q) c.c[q] = sd->c[q];
      // rows without tissue read the all-zero ghost brick and are not
      // stored: their values take no part in any tissue voxel's update (a
      // zero potential and stimulus give the same reaction value as the
      // stored rest state, and every weight coupling them is zero)
      const Cell q = cell_setup(nb, brick, rowm, ghost);
      const float v0 = gld(v, q.gl), w0 = gld(w, q.gl);
      const float j0 = jstim ? gld(jstim, q.gl) : 0.0f;
      float hv = 0.0f, hw = 0.0f, hj = 0.0f;
      if (q.has_halo) {
        hv = gld(v, q.hgl);
        hw = gld(w, q.hgl);
        hj = jstim ? gld(jstim, q.hgl) : 0.0f;
      }
      float k18[18];
      gather18(c, nb, brick, q.lx, q.ly, q.lz, k18, rowm, ghost, GLoad{});
      float vs, ws;
      ms_step(v0, w0, j0, ion, dt, vs, ws);
      s[q.C] = vs;
      if (q.has_halo) {
        float a, b;
        ms_step(hv, hw, hj, ion, dt, a, b);
        s[q.hC] = a;
      }
      __syncthreads();
      const float vn = vs + dt * apply19(s, q.C, k18);
      if (q.live) {
        gst(vout, q.g, vn);
        gst(wout, q.g, ws);
        if (v0 < theta && theta <= vn) {
          if (isinf(gld(tact, q.g)))
            gst(tact, q.g, static_cast<float>(tn) + dt * (theta - v0) / (vn - v0));
        }
        if (!isfinite(vn)) flags[0] = 1;
      }
    }
    it = it2;
    nbv = nbv2;
    rmv = rmv2;
    buf ^= 1;
  }
}

// after K substeps: step += K, clamped at the request's step count
__global__ void k_batch_advance(SlotDev* slots, int nslots, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots || !slots[i].active) return;
  const long long s = slots[i].step + K;
  slots[i].step = s < slots[i].n_steps ? s : slots[i].n_steps;
}

// first-fit allocator over one device allocation, coalescing on free
class Arena {
 public:
  void reset(size_t size) {
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  size_t alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return off;
      }
    }
    return std::numeric_limits<size_t>::max();
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

size_t region_bytes(const BrickMap& m) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(static_cast<size_t>(m.nb + 1) * kNbr * sizeof(int)) +
         al(static_cast<size_t>(m.nb + 1) * kNbr * sizeof(uint64_t)) +
         12 * al(static_cast<size_t>(m.nvox) * sizeof(float));
}

}  // namespace
}  // namespace ep

using namespace ep;

struct ep_batch_request {
  int64_t id = 0;
  int n[3] = {0, 0, 0};
  double h = 0, dt = 0, theta = 0.5;
  ep_ionic ionic{};
  // 3 fibre components per voxel and the scale (null: scale 1) in brick
  // layout, written on tissue only: the coefficient kernels never use the
  // values of other voxels, so the buffers are not cleared (clearing tens
  // of MB per request dominated the host cost of a submission)
  std::unique_ptr<double[]> fib_b;
  std::unique_ptr<double[]> scale_b;
  std::vector<int64_t> stim_idx; // stimulated voxels (brick layout) and their
  std::vector<double> stim_amp;  // summed amplitudes, same rule as the per-grid path
  double sig_l = 0, sig_t = 0;
  std::vector<ep_stim> stims;
  double t_on = 0, t_off = 0;
  int64_t n_steps = 0;
  BrickMap map;
  size_t bytes = 0, off = 0;
  int slot = -1;
  bool finished = false;
};

struct ep_batch_s {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t budget = 0;
  int max_slots = 0;
  int K = 1;
  char* arena_base = nullptr;
  Arena arena;
  size_t arena_peak = 0;
  SlotDev* d_slots = nullptr;
  SlotDev* h_slots = nullptr;   // pinned read-back of the slot table
  SlotDev* h_up = nullptr;      // pinned staging of slot uploads (one per slot, and a zero entry)
  hipStream_t rstream = nullptr;  // result reads (finished requests only)
  hipStream_t astream = nullptr;  // admissions (uploads and coefficient kernels)
  hipEvent_t ev_adm = nullptr;    // end of the admissions of an advance
  char* h_stage = nullptr;        // pinned upload staging: two halves of kStageHalf bytes
  hipEvent_t ev_stage[2] = {nullptr, nullptr};  // end of each half's copy
  bool stage_busy[2] = {false, false};
  int stage_next = 0;
  std::vector<int> unpublished;   // admitted slots not yet in the device slot table
  hipEvent_t ev_done = nullptr;   // end of the graph launch in flight
  bool inflight = false;
  std::vector<long long> launch_before;  // per slot: step at the launch in flight, -1 = not in it
  WorkItem* d_work = nullptr;
  int* d_count = nullptr;
  int* d_flags = nullptr;
  int work_cap = 0;
  // coefficient-encoding scratch (grown on demand)
  double* d_fib = nullptr;
  double* d_scale = nullptr;
  double* d_tens = nullptr;
  uint8_t* d_mask = nullptr;
  int64_t scratch_vox = 0;
  int64_t* d_stim_idx = nullptr;  // stimulus scatter scratch (grown on demand)
  double* d_stim_amp = nullptr;
  double* d_qstep = nullptr;
  size_t stim_cap = 0;
  WorkItem* h_work = nullptr;     // pinned staging of the work list (work_cap entries)
  int* h_count = nullptr;         // pinned staging of the work count
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraphNode_t> step_nodes;  // the K k_batch_step nodes of the graph
  int graph_blocks = 0;                    // their current grid size
  int work_count = 0;                      // length of the current work list
  std::deque<ep_batch_request*> queue;
  std::map<int64_t, ep_batch_request*> all;
  std::vector<int64_t> slot_owner;
  std::vector<int64_t> finished_ids;
  int64_t next_id = 1;
  ep_batch_stats st{};
  bool work_dirty = true;
  std::string err;
};

namespace {

ep_status bfail(ep_batch b, ep_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

#define BHIP(b, expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return bfail((b), EP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Upload of host data to the device on the admission stream, through the
// pinned staging halves: the host fills one half with all pool threads
// while the copy engine drains the other (a pageable copy would be staged
// by one host thread).  Returns once the last piece is enqueued; the source
// may be reused at once.
constexpr size_t kStageHalf = size_t(8) << 20;

ep_status upload(ep_batch b, void* dst, const void* src, size_t bytes) {
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  for (size_t off = 0; off < bytes; off += kStageHalf) {
    const size_t len = std::min(kStageHalf, bytes - off);
    const int h = b->stage_next;
    b->stage_next ^= 1;
    if (b->stage_busy[h]) BHIP(b, hipEventSynchronize(b->ev_stage[h]));
    char* st = b->h_stage + h * kStageHalf;
    constexpr size_t kPiece = size_t(256) << 10;
    const int64_t np = static_cast<int64_t>((len + kPiece - 1) / kPiece);
    parallel_for(np, [&](int64_t i) {
      const size_t o = static_cast<size_t>(i) * kPiece;
      std::memcpy(st + o, s + off + o, std::min(kPiece, len - o));
    });
    BHIP(b, hipMemcpyAsync(d + off, st, len, hipMemcpyHostToDevice, b->astream));
    BHIP(b, hipEventRecord(b->ev_stage[h], b->astream));
    b->stage_busy[h] = true;
  }
  return EP_OK;
}

ep_status grow_scratch(ep_batch b, int64_t nvox) {
  if (nvox <= b->scratch_vox) return EP_OK;
  BHIP(b, hipStreamSynchronize(b->astream));
  (void)hipFree(b->d_fib);
  (void)hipFree(b->d_scale);
  (void)hipFree(b->d_tens);
  (void)hipFree(b->d_mask);
  b->d_fib = b->d_scale = b->d_tens = nullptr;
  b->d_mask = nullptr;
  b->scratch_vox = 0;
  const size_t n = static_cast<size_t>(nvox);
  if (hipMalloc(&b->d_fib, 3 * n * sizeof(double)) != hipSuccess ||
      hipMalloc(&b->d_scale, n * sizeof(double)) != hipSuccess ||
      hipMalloc(&b->d_tens, 6 * n * sizeof(double)) != hipSuccess ||
      hipMalloc(&b->d_mask, n) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, EP_ERR_OOM, "coefficient scratch allocation failed");
  }
  b->scratch_vox = nvox;
  if (!b->d_qstep && hipMalloc(&b->d_qstep, sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, EP_ERR_OOM, "coefficient scratch allocation failed");
  }
  return EP_OK;
}

ep_status grow_stim(ep_batch b, size_t n) {
  if (n <= b->stim_cap) return EP_OK;
  BHIP(b, hipStreamSynchronize(b->astream));
  (void)hipFree(b->d_stim_idx);
  (void)hipFree(b->d_stim_amp);
  b->d_stim_idx = nullptr;
  b->d_stim_amp = nullptr;
  b->stim_cap = 0;
  if (hipMalloc(&b->d_stim_idx, n * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&b->d_stim_amp, n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, EP_ERR_OOM, "stimulus scratch allocation failed");
  }
  b->stim_cap = n;
  return EP_OK;
}

// Build a request's device region: weights, initial state, stimulus field.
// Everything is enqueued on the admission stream, so that it runs beside
// the graph launch in flight: the region was free (no launch in flight
// reads it), host data goes through the pinned staging halves, and the
// coefficient scratch is used by admissions only.
ep_status admit(ep_batch b, ep_batch_request* r, int slot) {
  const BrickMap& m = r->map;
  const size_t nv = static_cast<size_t>(m.nvox);
  const size_t nreal = static_cast<size_t>(m.nb) * kBV;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  char* base = b->arena_base + r->off;
  int* d_nbr = reinterpret_cast<int*>(base);
  char* p = base + al(static_cast<size_t>(m.nb + 1) * kNbr * sizeof(int));
  uint64_t* d_rowsn = reinterpret_cast<uint64_t*>(p);
  p += al(static_cast<size_t>(m.nb + 1) * kNbr * sizeof(uint64_t));
  float* arr[12];
  for (int k = 0; k < 12; ++k) {
    arr[k] = reinterpret_cast<float*>(p);
    p += al(nv * sizeof(float));
  }
  // arr: 0-5 weights, 6-7 v, 8-9 w, 10 tact, 11 jamp
  if (ep_status s = grow_scratch(b, m.nvox); s != EP_OK) return s;
  if (ep_status s = grow_stim(b, r->stim_idx.size()); s != EP_OK) return s;
  BHIP(b, hipMemsetAsync(base, 0, r->bytes, b->astream));
  // rest state on the real bricks (the ghost brick stays zero): w = 1 in
  // both buffers (rows without tissue are never stored), T_act = +inf
  BHIP(b, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(arr[8]), 0x3f800000u, nreal,
                            b->astream));
  BHIP(b, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(arr[9]), 0x3f800000u, nreal,
                            b->astream));
  BHIP(b, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(arr[10]), 0x7f800000u, nreal,
                            b->astream));
  if (ep_status s = upload(b, d_nbr, m.nbr.data(), m.nbr.size() * sizeof(int)); s != EP_OK)
    return s;
  if (ep_status s = upload(b, d_rowsn, m.rowsn.data(), m.rowsn.size() * sizeof(uint64_t));
      s != EP_OK)
    return s;
  if (ep_status s = upload(b, b->d_mask, m.mask.data(), nv); s != EP_OK) return s;
  if (ep_status s = upload(b, b->d_fib, r->fib_b.get(), 3 * nv * sizeof(double)); s != EP_OK)
    return s;
  if (r->scale_b)
    if (ep_status s = upload(b, b->d_scale, r->scale_b.get(), nv * sizeof(double)); s != EP_OK)
      return s;
  BHIP(b, hipMemsetAsync(b->d_tens, 0, 6 * nv * sizeof(double), b->astream));
  if (!r->stim_idx.empty()) {
    if (ep_status s = upload(b, b->d_stim_idx, r->stim_idx.data(),
                             r->stim_idx.size() * sizeof(int64_t));
        s != EP_OK)
      return s;
    if (ep_status s = upload(b, b->d_stim_amp, r->stim_amp.data(),
                             r->stim_amp.size() * sizeof(double));
        s != EP_OK)
      return s;
    launch_stim_scatter<float>(b->astream, b->d_stim_idx, b->d_stim_amp,
                               static_cast<int>(r->stim_idx.size()), arr[11], b->d_qstep);
  }
  LaunchCfg L;
  L.nb = m.nb;
  L.grid = grid_for(m.nb);
  L.pgrid = L.grid;
  L.stream = b->astream;
  L.rowsn = nullptr;
  float* c32[6];
  for (int k = 0; k < 6; ++k) c32[k] = arr[k];
  launch_tensor_coefs(L, d_nbr, b->d_mask, b->d_fib, r->scale_b ? b->d_scale : nullptr,
                      r->sig_l, r->sig_t, r->h, b->d_tens, nullptr, c32);
  BHIP(b, hipGetLastError());
  SlotDev& sd = b->h_up[slot];
  sd = SlotDev{};
  sd.nbr = d_nbr;
  sd.rowsn = d_rowsn;
  sd.nb = m.nb;
  for (int k = 0; k < 6; ++k) sd.c[k] = arr[k];
  sd.v[0] = arr[6];
  sd.v[1] = arr[7];
  sd.w[0] = arr[8];
  sd.w[1] = arr[9];
  sd.tact = arr[10];
  sd.jamp = r->stims.empty() ? nullptr : arr[11];
  sd.ion.inv_tau_in = static_cast<float>(1.0 / r->ionic.tau_in);
  sd.ion.inv_tau_out = static_cast<float>(1.0 / r->ionic.tau_out);
  sd.ion.inv_tau_open = static_cast<float>(1.0 / r->ionic.tau_open);
  sd.ion.inv_tau_close = static_cast<float>(1.0 / r->ionic.tau_close);
  sd.ion.v_gate = static_cast<float>(r->ionic.v_gate);
  sd.ion.exc = static_cast<float>(r->ionic.exc);
  sd.dt = static_cast<float>(r->dt);
  sd.theta = static_cast<float>(r->theta);
  sd.dtd = r->dt;
  sd.t_on = r->t_on;
  sd.t_off = r->t_off;
  sd.step = 0;
  sd.n_steps = r->n_steps;
  sd.active = 1;
  // the slot-table entry goes in after the launch in flight (publish_slot)
  r->slot = slot;
  b->slot_owner[slot] = r->id;
  b->st.admitted += 1;
  b->st.resident += 1;
  b->work_dirty = true;
  return EP_OK;
}

// Enter an admitted request into the slot table, from pinned staging that
// nothing rewrites before the copy has run.  Called after the wait for the
// launch in flight, whose last kernel advances every active slot and whose
// read-back overwrites the host copy of the table.
ep_status publish_slot(ep_batch b, int slot) {
  BHIP(b, hipMemcpyAsync(b->d_slots + slot, b->h_up + slot, sizeof(SlotDev),
                         hipMemcpyHostToDevice, b->stream));
  b->h_slots[slot] = b->h_up[slot];
  return EP_OK;
}

ep_status set_step_grid(ep_batch b);

// Grid of the captured step launches: persistent, as many blocks as stay
// resident (3 per CU at the step kernel's register use), or fewer for a
// short work list; a multiple of 8 (one share per XCD).
unsigned step_blocks(int work_count) {
  const int cap = 3 * 256;
  const int want = std::min(cap, std::max(1, work_count));
  return static_cast<unsigned>(((want + kXcd - 1) / kXcd) * kXcd);
}


// Work list of every running request's bricks.  Staged through pinned host
// memory and enqueued without waiting: the previous graph launch, which
// still reads the old list, runs first on the same stream, and the host
// never rewrites the staging area before the end of an advance, which
// waits for the stream.
ep_status rebuild_work(ep_batch b) {
  int64_t total = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    const int64_t id = b->slot_owner[s];
    if (id < 0) continue;
    const ep_batch_request* r = b->all[id];
    if (!r->finished) total += r->map.nb;
  }
  if (total > b->work_cap) {
    BHIP(b, hipStreamSynchronize(b->stream));
    (void)hipFree(b->d_work);
    (void)hipHostFree(b->h_work);
    b->d_work = nullptr;
    b->h_work = nullptr;
    b->work_cap = 0;
    void* hp = nullptr;
    if (hipMalloc(&b->d_work, total * sizeof(WorkItem)) != hipSuccess ||
        hipHostMalloc(&hp, total * sizeof(WorkItem), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, EP_ERR_OOM, "work list allocation failed");
    }
    b->h_work = static_cast<WorkItem*>(hp);
    b->work_cap = static_cast<int>(total);
    // the captured graph holds the old pointer: capture again
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (b->graph) {
      (void)hipGraphDestroy(b->graph);
      b->graph = nullptr;
    }
  }
  int n = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    const int64_t id = b->slot_owner[s];
    if (id < 0) continue;
    const ep_batch_request* r = b->all[id];
    if (r->finished) continue;
    for (int k = 0; k < r->map.nb; ++k) b->h_work[n++] = WorkItem{s, k};
  }
  *b->h_count = n;
  if (n) BHIP(b, hipMemcpyAsync(b->d_work, b->h_work, n * sizeof(WorkItem),
                                hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(b->d_count, b->h_count, sizeof(int), hipMemcpyHostToDevice, b->stream));
  b->work_count = n;
  b->work_dirty = false;
  // no launch is in flight here (the advance waited for it): resize the grid
  if (b->exec && b->graph_blocks != static_cast<int>(step_blocks(n)))
    if (ep_status s = set_step_grid(b); s != EP_OK) return s;
  return EP_OK;
}

ep_status set_step_grid(ep_batch b) {
  const unsigned blocks = step_blocks(b->work_count);
  for (hipGraphNode_t node : b->step_nodes) {
    hipKernelNodeParams kp{};
    BHIP(b, hipGraphKernelNodeGetParams(node, &kp));
    kp.gridDim = dim3(blocks);
    BHIP(b, hipGraphExecKernelNodeSetParams(b->exec, node, &kp));
  }
  b->graph_blocks = static_cast<int>(blocks);
  return EP_OK;
}

ep_status capture(ep_batch b) {
  if (b->exec) return EP_OK;
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const unsigned blocks = step_blocks(b->work_count);
  for (int k = 0; k < b->K; ++k)
    k_batch_step<<<blocks, kBV, 0, b->stream>>>(b->d_slots, b->d_work, b->d_count, k, b->d_flags);
  k_batch_advance<<<(b->max_slots + 255) / 256, 256, 0, b->stream>>>(b->d_slots, b->max_slots,
                                                                     b->K);
  hipGraph_t gr = nullptr;
  BHIP(b, hipStreamEndCapture(b->stream, &gr));
  b->graph = gr;
  BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->graph_blocks = static_cast<int>(blocks);
  // the K step-kernel nodes, for later grid updates
  size_t nn = 0;
  BHIP(b, hipGraphGetNodes(b->graph, nullptr, &nn));
  std::vector<hipGraphNode_t> nodes(nn);
  BHIP(b, hipGraphGetNodes(b->graph, nodes.data(), &nn));
  b->step_nodes.clear();
  for (hipGraphNode_t node : nodes) {
    hipGraphNodeType ty;
    BHIP(b, hipGraphNodeGetType(node, &ty));
    if (ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    BHIP(b, hipGraphKernelNodeGetParams(node, &kp));
    if (kp.func == reinterpret_cast<void*>(&k_batch_step)) b->step_nodes.push_back(node);
  }
  if (static_cast<int>(b->step_nodes.size()) != b->K)
    return bfail(b, EP_ERR_HIP, "captured graph does not hold the expected step launches");
  return EP_OK;
}

}  // namespace

extern "C" {

EP_API ep_status ep_batch_create(const ep_batch_desc* d, ep_batch* out) {
  if (!out) return EP_ERR_ARG;
  *out = nullptr;
  if (!d || d->hbm_budget <= 0 || d->max_slots < 1 || d->steps_per_launch < 1)
    return EP_ERR_ARG;
  ep_batch b = new (std::nothrow) ep_batch_s();
  if (!b) return EP_ERR_OOM;
  b->budget = d->hbm_budget;
  b->max_slots = d->max_slots;
  b->K = d->steps_per_launch;
  ep_status s = EP_OK;
  do {
    if (d->stream) {
      b->stream = static_cast<hipStream_t>(d->stream);
    } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess) {
      b->own_stream = true;
    } else {
      s = EP_ERR_HIP;
      break;
    }
    if (hipMalloc(&b->arena_base, static_cast<size_t>(b->budget)) != hipSuccess ||
        hipMalloc(&b->d_slots, b->max_slots * sizeof(SlotDev)) != hipSuccess ||
        hipMalloc(&b->d_count, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->d_flags, 4 * sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      s = EP_ERR_OOM;
      break;
    }
    void* hp = nullptr;
    if (hipHostMalloc(&hp, b->max_slots * sizeof(SlotDev), hipHostMallocDefault) != hipSuccess) {
      s = EP_ERR_OOM;
      break;
    }
    b->h_slots = static_cast<SlotDev*>(hp);
    std::memset(b->h_slots, 0, b->max_slots * sizeof(SlotDev));
    void* hu = nullptr;
    if (hipHostMalloc(&hu, (b->max_slots + 1) * sizeof(SlotDev), hipHostMallocDefault) !=
        hipSuccess) {
      s = EP_ERR_OOM;
      break;
    }
    b->h_up = static_cast<SlotDev*>(hu);
    std::memset(b->h_up, 0, (b->max_slots + 1) * sizeof(SlotDev));
    void* hs = nullptr;
    if (hipHostMalloc(&hs, 2 * kStageHalf, hipHostMallocDefault) != hipSuccess) {
      s = EP_ERR_OOM;
      break;
    }
    b->h_stage = static_cast<char*>(hs);
    if (hipStreamCreateWithFlags(&b->rstream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->astream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_adm, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_stage[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_stage[1], hipEventDisableTiming) != hipSuccess) {
      s = EP_ERR_HIP;
      break;
    }
    b->launch_before.assign(b->max_slots, -1);
    if (hipMemsetAsync(b->d_slots, 0, b->max_slots * sizeof(SlotDev), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_count, 0, sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_flags, 0, 4 * sizeof(int), b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
      s = EP_ERR_HIP;
      break;
    }
    b->arena.reset(static_cast<size_t>(b->budget));
    b->slot_owner.assign(b->max_slots, -1);
    // every resident brick holds at least 12 arrays of 512 floats of arena,
    // so this many work items always suffice
    b->work_cap = static_cast<int>(b->budget / (12 * kBV * sizeof(float))) + b->max_slots;
    void* hw = nullptr;
    void* hc = nullptr;
    if (hipMalloc(&b->d_work, static_cast<size_t>(b->work_cap) * sizeof(WorkItem)) != hipSuccess ||
        hipHostMalloc(&hw, static_cast<size_t>(b->work_cap) * sizeof(WorkItem),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&hc, sizeof(int), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      s = EP_ERR_OOM;
      break;
    }
    b->h_work = static_cast<WorkItem*>(hw);
    b->h_count = static_cast<int*>(hc);
  } while (false);
  if (s != EP_OK) {
    ep_batch_destroy(b);
    return s;
  }
  *out = b;
  return EP_OK;
}

EP_API ep_status ep_batch_submit(ep_batch b, const ep_grid_desc* d, const double* fibre,
                                 const double* scale, double sig_l, double sig_t,
                                 int64_t n_steps, int64_t* id) {
  if (!b) return EP_ERR_ARG;
  if (!d || !fibre || !id || n_steps < 0) return bfail(b, EP_ERR_ARG, "bad submit arguments");
  if (d->model != EP_MONO || d->prec != EP_F32 || d->diff != EP_DIFF_EXPLICIT)
    return bfail(b, EP_ERR_UNSUPPORTED, "batched serving runs FP32 explicit monodomain only");
  for (int k = 0; k < 3; ++k)
    if (d->n[k] < 1 || d->n[k] > 4096) return bfail(b, EP_ERR_ARG, "n must be in [1, 4096]");
  if (!(d->h > 0) || !(d->dt > 0) || !(d->act_threshold > 0 && d->act_threshold < 1))
    return bfail(b, EP_ERR_ARG, "bad h, dt or threshold");
  const ep_ionic& io = d->ionic;
  if (!(io.tau_in > 0) || !(io.tau_out > 0) || !(io.tau_open > 0) || !(io.tau_close > 0) ||
      !(io.exc >= 0))
    return bfail(b, EP_ERR_ARG, "ionic time constants must be > 0 and exc >= 0");
  if (!(sig_l >= 0) || !(sig_t >= 0) || !std::isfinite(sig_l) || !std::isfinite(sig_t))
    return bfail(b, EP_ERR_ARG, "conductivities must be finite and >= 0");
  if (d->n_stim < 0 || (d->n_stim > 0 && !d->stim)) return bfail(b, EP_ERR_ARG, "bad stimuli");
  try {
    auto* r = new ep_batch_request();
    std::unique_ptr<ep_batch_request> guard(r);
    std::copy(d->n, d->n + 3, r->n);
    r->h = d->h;
    r->dt = d->dt;
    r->theta = d->act_threshold;
    r->ionic = d->ionic;
    r->sig_l = sig_l;
    r->sig_t = sig_t;
    r->n_steps = n_steps;
    r->stims.assign(d->stim, d->stim + d->n_stim);
    for (size_t k = 0; k < r->stims.size(); ++k)
      if (r->stims[k].t_on != r->stims[0].t_on || r->stims[k].t_off != r->stims[0].t_off)
        return bfail(b, EP_ERR_UNSUPPORTED, "stimuli of a batched request share one window");
    if (!r->stims.empty()) {
      r->t_on = r->stims[0].t_on;
      r->t_off = r->stims[0].t_off;
    }
    std::string merr;
    if (!build_brick_map(r->n, d->mask, r->map, merr)) return bfail(b, EP_ERR_ARG, merr);
    const BrickMap& m = r->map;
    const size_t nv = static_cast<size_t>(m.nvox);
    if (m.nvox > (int64_t(1) << 29))
      return bfail(b, EP_ERR_UNSUPPORTED, "request too large: more than 2^29 voxels in active bricks");
    // fibres (and scale) to brick layout, validated on tissue
    r->fib_b.reset(new double[3 * nv]);
    if (scale) r->scale_b.reset(new double[nv]);
    std::atomic<int> bad{0};   // 1: non-unit fibre, 2: bad scale
    std::vector<double> smax_b(m.nb, 0.0);
    // one brick per task: its tissue rows are short contiguous runs of the
    // box-layout input and one contiguous block of the output
    parallel_for(m.nb, [&](int64_t id) {
      const int bx = m.brick_pos[3 * id], by = m.brick_pos[3 * id + 1],
                bz = m.brick_pos[3 * id + 2];
      const uint64_t rows = m.rows[id];
      double sm = 0.0;
      for (int row = 0; row < 64; ++row) {
        if (!((rows >> row) & 1)) continue;
        const int x = 8 * bx + (row >> 3), y = 8 * by + (row & 7);
        for (int lz = 0; lz < 8; ++lz) {
          const int z = 8 * bz + lz;
          if (z >= r->n[2]) break;
          const int64_t gi = id * kBV + row * 8 + lz;
          if (!m.mask[gi]) continue;
          const int64_t bi = m.box_index(x, y, z);
          const double f0 = fibre[3 * bi], f1 = fibre[3 * bi + 1], f2 = fibre[3 * bi + 2];
          if (!(std::fabs(std::sqrt(f0 * f0 + f1 * f1 + f2 * f2) - 1.0) <= 1e-6)) bad.store(1);
          r->fib_b[3 * gi] = f0;
          r->fib_b[3 * gi + 1] = f1;
          r->fib_b[3 * gi + 2] = f2;
          if (scale) {
            if (!(scale[bi] > 0) || !std::isfinite(scale[bi])) bad.store(2);
            r->scale_b[gi] = scale[bi];
            sm = std::max(sm, scale[bi]);
          }
        }
      }
      smax_b[id] = sm;
    });
    if (bad.load() == 1) return bfail(b, EP_ERR_ARG, "fibre is not a unit vector on a tissue voxel");
    if (bad.load() == 2) return bfail(b, EP_ERR_ARG, "scale must be finite and > 0 on tissue");
    double smax = 1.0;
    if (scale) smax = *std::max_element(smax_b.begin(), smax_b.end());
    // stimulated voxels with their summed amplitudes (stimuli in order, as
    // the per-grid path sums them)
    std::vector<std::pair<int64_t, double>> sv;
    for (const ep_stim& st : r->stims)
      for (int x = std::max(0, st.lo[0]); x < std::min(r->n[0], st.hi[0]); ++x)
        for (int y = std::max(0, st.lo[1]); y < std::min(r->n[1], st.hi[1]); ++y)
          for (int z = std::max(0, st.lo[2]); z < std::min(r->n[2], st.hi[2]); ++z) {
            const int64_t gi = m.brick_index(x, y, z);
            if (gi < 0 || !m.mask[gi]) continue;
            if (st.radius > 0.0) {
              const double dx = (x + 0.5) * r->h - st.center[0];
              const double dy = (y + 0.5) * r->h - st.center[1];
              const double dz = (z + 0.5) * r->h - st.center[2];
              const double r2 = dx * dx + dy * dy + dz * dz;
              if (!(r2 <= st.radius * st.radius)) continue;
            }
            sv.emplace_back(gi, st.amp);
          }
    std::stable_sort(sv.begin(), sv.end(),
                     [](const auto& a, const auto& c) { return a.first < c.first; });
    for (size_t k = 0; k < sv.size();) {
      double acc = 0.0;
      size_t e = k;
      for (; e < sv.size() && sv[e].first == sv[k].first; ++e) acc += sv[e].second;
      r->stim_idx.push_back(sv[k].first);
      r->stim_amp.push_back(acc);
      k = e;
    }
    // explicit stability, conservatively: |A_pp| + sum_q |A_pq| <=
    // 4 smax (sig_l + 2 sig_t + |sig_l - sig_t|) / h^2 for unit fibres
    const double gb = 4.0 * smax * (sig_l + 2.0 * sig_t + std::fabs(sig_l - sig_t)) / (r->h * r->h);
    if (!(r->dt * gb < 2.0))
      return bfail(b, EP_ERR_ARG, "explicit diffusion may be unstable for this dt (bound test)");
    r->bytes = region_bytes(r->map);
    if (static_cast<int64_t>(r->bytes) > b->budget)
      return bfail(b, EP_ERR_OOM, "request larger than the batch's HBM budget");
    r->id = b->next_id++;
    guard.release();
    b->all[r->id] = r;
    b->queue.push_back(r);
    b->st.submitted += 1;
    b->st.queued = static_cast<int32_t>(b->queue.size());
    *id = r->id;
    return EP_OK;
  } catch (const std::bad_alloc&) {
    return bfail(b, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_batch_advance(ep_batch b, int32_t* n_finished) {
  if (!b) return EP_ERR_ARG;
  try {
    // admission, FIFO while memory and a slot are free, before the wait:
    // the uploads and coefficient kernels run beside the launch in flight
    // (slots and regions freed by releases are not in its work list)
    while (!b->queue.empty()) {
      ep_batch_request* r = b->queue.front();
      int slot = -1;
      for (int s = 0; s < b->max_slots; ++s)
        if (b->slot_owner[s] < 0) { slot = s; break; }
      if (slot < 0) break;
      const size_t off = b->arena.alloc(r->bytes);
      if (off == std::numeric_limits<size_t>::max()) break;
      r->off = off;
      b->queue.pop_front();
      if (ep_status s = admit(b, r, slot); s != EP_OK) {
        // back to the head of the queue with its region freed, for a later
        // advance to try again (what the failed admission enqueued into the
        // region runs before any later admission's, on the same stream)
        b->arena.release(off, r->bytes);
        b->queue.push_front(r);
        b->st.queued = static_cast<int32_t>(b->queue.size());
        return s;
      }
      b->unpublished.push_back(slot);
      b->arena_peak = std::max(b->arena_peak, b->arena.used());
    }
    b->st.queued = static_cast<int32_t>(b->queue.size());
    if (!b->unpublished.empty()) {
      // the next launch runs after the admissions
      BHIP(b, hipEventRecord(b->ev_adm, b->astream));
      BHIP(b, hipStreamWaitEvent(b->stream, b->ev_adm, 0));
    }
    // results of the graph launch in flight: wait for it, read the slot table
    int nfin = 0;
    if (b->inflight) {
      BHIP(b, hipEventSynchronize(b->ev_done));
      b->inflight = false;
      for (int s = 0; s < b->max_slots; ++s) {
        if (b->launch_before[s] < 0) continue;
        const int64_t id = b->slot_owner[s];
        ep_batch_request* r = b->all[id];
        b->st.voxel_steps += static_cast<double>(b->h_slots[s].step - b->launch_before[s]) *
                             static_cast<double>(r->map.n_tissue);
        b->launch_before[s] = -1;
        if (b->h_slots[s].step >= r->n_steps) {
          r->finished = true;
          b->finished_ids.push_back(id);
          b->st.finished += 1;
          b->work_dirty = true;
          ++nfin;
        }
      }
    }
    const bool admitted = !b->unpublished.empty();
    for (int slot : b->unpublished)
      if (ep_status s = publish_slot(b, slot); s != EP_OK) return s;
    b->unpublished.clear();
    if (b->work_dirty)
      if (ep_status s = rebuild_work(b); s != EP_OK) return s;
    if (ep_status s = capture(b); s != EP_OK) return s;
    // one graph launch of K steps for every running request, three after
    // an admission (the host goes on building requests meanwhile, and short
    // launches would leave the device idle); the host returns at once and
    // collects the results at the next call.  A slot that reaches its step
    // count in one launch is skipped by the later ones.
    bool any = false;
    for (int s = 0; s < b->max_slots; ++s) {
      const int64_t id = b->slot_owner[s];
      if (id >= 0 && !b->all[id]->finished) {
        b->launch_before[s] = b->h_slots[s].step;
        any = true;
      }
    }
    if (any) {
      for (int l = 0; l < (admitted ? 3 : 1); ++l) {
        BHIP(b, hipGraphLaunch(b->exec, b->stream));
        b->st.graph_launches += 1;
      }
      BHIP(b, hipMemcpyAsync(b->h_slots, b->d_slots, b->max_slots * sizeof(SlotDev),
                             hipMemcpyDeviceToHost, b->stream));
      BHIP(b, hipEventRecord(b->ev_done, b->stream));
      b->inflight = true;
    }
    if (n_finished) *n_finished = nfin;
    return EP_OK;
  } catch (const std::bad_alloc&) {
    return bfail(b, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_batch_finished(ep_batch b, int64_t* ids, int32_t cap, int32_t* n) {
  if (!b || !n || (cap > 0 && !ids)) return EP_ERR_ARG;
  const int32_t k = static_cast<int32_t>(std::min<size_t>(cap, b->finished_ids.size()));
  for (int32_t i = 0; i < k; ++i) ids[i] = b->finished_ids[i];
  b->finished_ids.erase(b->finished_ids.begin(), b->finished_ids.begin() + k);
  *n = k;
  return EP_OK;
}

EP_API ep_status ep_batch_read(ep_batch b, int64_t id, ep_field f, double* host_out, size_t n) {
  if (!b || !host_out) return EP_ERR_ARG;
  auto it = b->all.find(id);
  if (it == b->all.end()) return bfail(b, EP_ERR_ARG, "unknown request id");
  ep_batch_request* r = it->second;
  if (r->slot < 0) return bfail(b, EP_ERR_STATE, "request not admitted yet");
  if (f != EP_V && f != EP_W && f != EP_TACT) return bfail(b, EP_ERR_ARG, "bad field");
  const BrickMap& m = r->map;
  const size_t N = static_cast<size_t>(r->n[0]) * r->n[1] * r->n[2];
  if (n < N) return bfail(b, EP_ERR_ARG, "output buffer too small");
  try {
    // A finished request's buffers are no longer touched by any launch (it
    // left the work list before the launch in flight): read them on the
    // read stream, concurrently with that launch.  A running request is read
    // after the launch in flight.
    int64_t step = r->n_steps;
    hipStream_t rs = b->rstream;
    if (!r->finished) {
      BHIP(b, hipStreamSynchronize(b->astream));
      BHIP(b, hipStreamSynchronize(b->stream));
      SlotDev cur{};
      if (std::find(b->unpublished.begin(), b->unpublished.end(), r->slot) ==
          b->unpublished.end())
        BHIP(b, hipMemcpy(&cur, b->d_slots + r->slot, sizeof(SlotDev), hipMemcpyDeviceToHost));
      step = cur.step;   // 0 for a request that no launch has stepped yet
      rs = b->stream;
    }
    const SlotDev& sd = b->h_up[r->slot];   // the request's buffer pointers
    const int par = static_cast<int>(step & 1);
    const float* src = f == EP_V ? sd.v[par] : (f == EP_W ? sd.w[par] : sd.tact);
    std::vector<float> buf(m.nvox);
    BHIP(b, hipMemcpyAsync(buf.data(), src, m.nvox * sizeof(float), hipMemcpyDeviceToHost, rs));
    BHIP(b, hipStreamSynchronize(rs));
    const double off = f == EP_TACT ? std::numeric_limits<double>::infinity() : 0.0;
    parallel_for(r->n[0], [&](int64_t xx) {
      const int x = static_cast<int>(xx);
      for (int y = 0; y < r->n[1]; ++y)
        for (int z = 0; z < r->n[2]; ++z) {
          const int64_t gi = m.brick_index(x, y, z);
          host_out[m.box_index(x, y, z)] =
              (gi >= 0 && m.mask[gi]) ? static_cast<double>(buf[gi]) : off;
        }
    });
    return EP_OK;
  } catch (const std::bad_alloc&) {
    return bfail(b, EP_ERR_OOM, "host allocation failed");
  }
}

EP_API ep_status ep_batch_release(ep_batch b, int64_t id) {
  if (!b) return EP_ERR_ARG;
  auto it = b->all.find(id);
  if (it == b->all.end()) return bfail(b, EP_ERR_ARG, "unknown request id");
  ep_batch_request* r = it->second;
  if (r->slot >= 0) {
    if (!r->finished) {
      // still in the work list of the launch in flight, or being admitted:
      // let both end first
      BHIP(b, hipStreamSynchronize(b->astream));
      BHIP(b, hipStreamSynchronize(b->stream));
      b->launch_before[r->slot] = -1;
      b->unpublished.erase(std::remove(b->unpublished.begin(), b->unpublished.end(), r->slot),
                           b->unpublished.end());
    }
    // clear the slot after the launch in flight (the zero entry of the
    // pinned staging area is never written)
    BHIP(b, hipMemcpyAsync(b->d_slots + r->slot, b->h_up + b->max_slots, sizeof(SlotDev),
                           hipMemcpyHostToDevice, b->stream));
    b->arena.release(r->off, r->bytes);
    b->slot_owner[r->slot] = -1;
    b->st.resident -= 1;
    b->work_dirty = true;
  } else {
    b->queue.erase(std::remove(b->queue.begin(), b->queue.end(), r), b->queue.end());
    b->st.queued = static_cast<int32_t>(b->queue.size());
  }
  b->finished_ids.erase(std::remove(b->finished_ids.begin(), b->finished_ids.end(), id),
                        b->finished_ids.end());
  b->st.released += 1;
  b->all.erase(it);
  delete r;
  return EP_OK;
}

EP_API ep_status ep_batch_get_stats(ep_batch b, ep_batch_stats* s) {
  if (!b || !s) return EP_ERR_ARG;
  *s = b->st;
  s->arena_used = static_cast<int64_t>(b->arena.used());
  s->arena_peak = static_cast<int64_t>(b->arena_peak);
  return EP_OK;
}

EP_API ep_status ep_batch_destroy(ep_batch b) {
  if (!b) return EP_ERR_ARG;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->astream) (void)hipStreamSynchronize(b->astream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& kv : b->all) delete kv.second;
  (void)hipFree(b->arena_base);
  (void)hipFree(b->d_slots);
  (void)hipFree(b->d_work);
  (void)hipFree(b->d_count);
  (void)hipFree(b->d_flags);
  (void)hipFree(b->d_fib);
  (void)hipFree(b->d_scale);
  (void)hipFree(b->d_tens);
  (void)hipFree(b->d_mask);
  (void)hipFree(b->d_stim_idx);
  (void)hipFree(b->d_stim_amp);
  (void)hipFree(b->d_qstep);
  if (b->h_slots) (void)hipHostFree(b->h_slots);
  if (b->h_up) (void)hipHostFree(b->h_up);
  if (b->ev_done) (void)hipEventDestroy(b->ev_done);
  if (b->ev_adm) (void)hipEventDestroy(b->ev_adm);
  for (hipEvent_t e : b->ev_stage)
    if (e) (void)hipEventDestroy(e);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  if (b->rstream) (void)hipStreamDestroy(b->rstream);
  if (b->astream) (void)hipStreamDestroy(b->astream);
  if (b->h_work) (void)hipHostFree(b->h_work);
  if (b->h_count) (void)hipHostFree(b->h_count);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return EP_OK;
}

EP_API const char* ep_batch_last_error(ep_batch b) { return b ? b->err.c_str() : ""; }

}  // extern "C"

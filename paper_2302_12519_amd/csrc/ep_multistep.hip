// Several explicit monodomain steps in one launch, for grids small enough
// that every brick has a resident workgroup (a few hundred bricks).
//
// Such a grid moves a few MB per step, so one launch per step is bound by
// the launch and by the dependent load chain of each launch (neighbour table,
// then halo and weights, then the tile), not by HBM.  Here each workgroup
// keeps its brick's state (v, w, T_act), its 18 operator weights and its
// neighbour table in registers and LDS for the whole run, and a step costs
// one exchange of the post-reaction potential v* through a ping-pong pair of
// global arrays plus one grid-wide barrier:
//   reaction (registers) -> store own v* -> barrier -> load the 480 halo
//   cells of v* -> LDS tile -> 19-point diffusion -> activation check.
// The arithmetic is the per-step kernel's (k_explicit): the same reaction
// and operator code on the same values, so the two paths agree bitwise.
//
// The launch is cooperative (hipLaunchCooperativeKernel), which guarantees
// that all workgroups are resident at once, so the barrier cannot wait on a
// workgroup that never starts.  Its spin is bounded all the same: past the
// limit a workgroup records the timeout in flags[2] and leaves; every other
// workgroup then leaves at that barrier or the next, so the launch always
// ends, and the host reports the error.
#include <hip/hip_runtime.h>

#include "ep_device.h"

namespace ep {
namespace {

using namespace dev;

// about 10^6 polls of a few hundred ns: far beyond any legitimate wait
constexpr unsigned kSpinLimit = 1u << 20;

// Barrier number k of the launch completes when the arrival counter reaches
// (k + 1) * gridDim.x (the counter is zero at launch).  What crosses it is
// only the exchanged v*, written and read with agent-scope accesses that go
// to the device-coherent level (see put_agent / get_agent), so no cache
// write-back or invalidation is needed: every thread waits until its own
// store is acknowledged there, the workgroup meets, thread 0 arrives and
// polls the counter, and the workgroup meets again before any halo load is
// issued.  Returns false (in every thread) when the wait timed out.
__device__ __forceinline__ bool grid_barrier(unsigned* count, unsigned target, int* flags) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > kSpinLimit) {
        good = 0;
        __hip_atomic_fetch_or(&flags[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Stores and loads of the exchanged v* bypass the caches that are not
// coherent across XCDs (agent-scope atomic accesses), so a halo load never
// sees a line another XCD's L2 kept from two steps earlier.
template <typename T>
__device__ __forceinline__ void put_agent(T* base, int i, T x) {
  __hip_atomic_store(&at(base, i), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T get_agent(T* base, int i) {
  return __hip_atomic_load(&at(base, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// nsteps explicit steps t_n, n = step0 .. step0 + nsteps - 1, with one
// stimulus field (jstim, nullable) for all of them.  vin/win may alias
// vout/wout: each thread reads its own voxel before the first barrier and
// writes it after the last.  xa, xb: exchange arrays of (nb + 1) * 512
// values whose ghost brick (index nb) holds zeros.  qstep (nullable): the
// stimulus charge rate, added nsteps times to qacc by one thread.
template <typename T>
__global__ __launch_bounds__(kBV) void k_explicit_ms(
    int nb, const int* __restrict__ nbr, CoefSet<T> c, const T* vin, const T* win,
    const T* __restrict__ jstim, T* vout, T* wout, T* __restrict__ tact, T* xa, T* xb,
    IonicT<T> ion, T dt, T theta, double dt64, long long step0, int nsteps, double* qacc,
    const double* qstep, double qscale, unsigned* count, int* flags) {
  __shared__ T s[kTile];
  __shared__ int nbs[kNbr];
  const int brick = blockIdx.x;
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  T v = at(vin, q.g), w = at(win, q.g);
  const T j = jstim ? at(jstim, q.g) : T(0);
  T ta = at(tact, q.g);
  bool crossed = false, bad = false;
  T k18[18];
  gather18(c, nbs, brick, q.lx, q.ly, q.lz, k18);
  for (int k = 0; k < nsteps; ++k) {
    T vs, ws;
    ms_step(v, w, j, ion, dt, vs, ws);
    T* x = (k & 1) ? xb : xa;
    put_agent(x, q.g, vs);
    if (!grid_barrier(count, static_cast<unsigned>(k + 1) * static_cast<unsigned>(nb), flags))
      return;
    s[q.C] = vs;
    if (q.has_halo) s[q.hC] = get_agent(x, q.hg);
    __syncthreads();
    const T vn = vs + dt * apply19(s, q.C, k18);
    if (v < theta && theta <= vn && isinf(ta)) {
      // t_n rounded on its own, as the per-step kernel receives it (no
      // fused multiply-add of n * dt into the sum)
#pragma clang fp contract(off)
      const double tn = static_cast<double>(step0 + k) * dt64;
      ta = static_cast<T>(tn) + dt * (theta - v) / (vn - v);
      crossed = true;
    }
    bad = bad || !isfinite(vn);
    v = vn;
    w = ws;
  }
  at(vout, q.g) = v;
  at(wout, q.g) = w;
  if (crossed) at(tact, q.g) = ta;
  if (bad) flags[0] = 1;
  if (qstep && blockIdx.x == 0 && threadIdx.x == 0) {
    // the per-step launches' additions, in registers: each is one fused
    // multiply-add, as k_q_accum compiles to
    const double q0 = qstep[0];
    double a = qacc[0];
    for (int k = 0; k < nsteps; ++k) a = fma(qscale, q0, a);
    qacc[0] = a;
  }
}

template <typename T>
const void* ms_kernel() {
  return reinterpret_cast<const void*>(&k_explicit_ms<T>);
}

}  // namespace

template <typename T>
int explicit_ms_capacity() {
  int dev = 0, cus = 0, coop = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, ms_kernel<T>(), kBV, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return coop ? per * cus : 0;
}

template <typename T>
hipError_t launch_explicit_ms(hipStream_t st, int nb, const int* nbr, CoefSet<T> c,
                              const T* vin, const T* win, const T* jstim, T* vout, T* wout,
                              T* tact, T* xa, T* xb, IonicT<T> ion, T dt, T theta, double dt64,
                              long long step0, int nsteps, double* qacc, const double* qstep,
                              double qscale, unsigned* count, int* flags) {
  hipError_t e = hipMemsetAsync(count, 0, sizeof(unsigned), st);
  if (e != hipSuccess) return e;
  void* args[] = {&nb,   &nbr,   &c,    &vin,  &win,   &jstim, &vout,   &wout,
                  &tact, &xa,    &xb,   &ion,  &dt,    &theta, &dt64,   &step0,
                  &nsteps, &qacc, &qstep, &qscale, &count, &flags};
  return hipLaunchCooperativeKernel(ms_kernel<T>(), dim3(nb), dim3(kBV), args, 0, st);
}

#define EP_MS_INST(T)                                                                          \
  template int explicit_ms_capacity<T>();                                                      \
  template hipError_t launch_explicit_ms<T>(hipStream_t, int, const int*, CoefSet<T>,          \
                                            const T*, const T*, const T*, T*, T*, T*, T*, T*,  \
                                            IonicT<T>, T, T, double, long long, int, double*,  \
                                            const double*, double, unsigned*, int*);
EP_MS_INST(float)
EP_MS_INST(double)
#undef EP_MS_INST

}  // namespace ep

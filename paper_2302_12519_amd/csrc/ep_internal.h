// Internal declarations of the HIP voxel-EP library (not part of the ABI).
//
// Data layout in HBM.  The box is cut into 8x8x8 bricks; only bricks that
// hold at least one tissue voxel are stored ("active" bricks, ids 0..nb-1 in
// x-major brick order), followed by one all-zero "ghost" brick (id nb) that
// stands in for every missing neighbour.  Inside a brick the 512 voxels are
// z-fastest: local index l = (lx*8 + ly)*8 + lz, so one 64-lane wavefront
// reads one x-plane of a brick as 256 contiguous bytes (FP32).  Every
// per-voxel array (state, coefficients, CG vectors) is (nb+1)*512 long and
// indexed brick*512 + l.  A neighbour table nbr[(nb+1)*27] maps each brick
// and offset (dx,dy,dz) in {-1,0,1}^3 to a brick id (ghost when absent).
//
// Non-tissue voxels inside active bricks hold v = 0, w = 1 (the ionic rest
// point, a bitwise fixed point of the update) and every stencil coefficient
// touching them is zero, so kernels need no mask on the hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ep {

constexpr int kB = 8;         // brick edge
constexpr int kBV = 512;      // voxels per brick
constexpr int kH = 10;        // brick edge plus a one-voxel halo on each side
constexpr int kTile = 1000;   // kH^3
constexpr int kHalo = 480;    // face (6x64) + edge (12x8) halo cells; corners unused
constexpr int kNbr = 27;
constexpr int kXcd = 8;       // MI355X: 8 accelerator complex dies
constexpr int kRedThreads = 1024;

// Coefficient slots of the 19-point operator, per voxel p:
//   CX, CY, CZ: face weight between p and p+e_d, Dface_dd / h^2
//   CXY, CXZ, CYZ: edge weight of the 2x2 block whose lower corner is p,
//                 Dedge_dd' / (2 h^2)
enum { CX = 0, CY = 1, CZ = 2, CXY = 3, CXZ = 4, CYZ = 5 };

template <typename T>
struct IonicT {
  T inv_tau_in, inv_tau_out, inv_tau_open, inv_tau_close, v_gate, exc;
};

template <typename T>
struct CoefSet {
  const T* c[6];
};

template <typename T>
struct CoefOut {
  T* c[6];
};

// Device-resident scalars of one CG solve.  Every CG kernel reads `done`
// first and returns at once when it is set, so a fixed sequence of launches
// can be enqueued without a host round trip per iteration.
struct CGScalars {
  double rz;      // (r, M^-1 r)
  double pq;      // (p, K p)
  double rr;      // (r, r)
  double bb;      // (b, b) (or the initial (r, r) for refinement inner solves)
  double tol2;    // rtol^2
  double alpha, beta;
  double rsum;    // sum of r over tissue (elliptic gauge)
  int it, maxit, done, fail;
};

struct LaunchCfg {
  int nb;       // active bricks
  int grid;     // blocks of a one-brick-per-block launch (multiple of kXcd, >= nb)
  int pgrid;    // blocks of a persistent launch (multiple of kXcd, <= grid)
  hipStream_t stream;
  const uint64_t* rowsn;   // (nb+1)*27 row masks of each brick's neighbourhood
  bool stream_nt = false;  // implicit-step kernels: non-temporal own-voxel streams
};

// The implicit step touches about 24 state-precision arrays per step.  Once
// they exceed the last-level cache (256 MB on MI355X), the kernels mark the
// accesses no other brick reads as non-temporal.
constexpr int kBeArrays = 24;
constexpr long long kLlcBytes = 256ll << 20;

inline int grid_for(int nb) { return ((nb + kXcd - 1) / kXcd) * kXcd; }
// persistent launches: as many 512-thread blocks as stay resident on the
// 256 CUs (the persistent CG kernels need 100-115 VGPRs: 2 blocks per CU)
inline int pgrid_for(int nb, bool /*fp64*/) {
  const int g = grid_for(nb);
  return g < 512 ? g : 512;
}
// ---- kernel launchers (ep_kernels.hip) ----------------------------------
// 19-point weights of the voxel tensors on mask; with body (elliptic domain
// with a bath, nullable) the weights cover body, whose non-tissue voxels
// carry sig_body I
void launch_tensor_coefs(const LaunchCfg& L, const int* nbr, const uint8_t* mask,
                         const double* fib, const double* scale, double sig_l, double sig_t,
                         double h, double* tens /*6 arrays, scratch*/, double* c64[6],
                         float* c32[6], const uint8_t* body = nullptr, double sig_body = 0.0);

// acc += add over every active brick, and out32 = (float) acc
void launch_coef_add(const LaunchCfg& L, double* const acc[6], double* const add[6],
                     float* const out32[6]);

// corner tensors of the corner-gradient operator A27 (one corner per voxel,
// the six entries in the slots CX..CYZ read as xx, yy, zz, xy, xz, yz)
void launch_corner_coefs(const LaunchCfg& L, const int* nbr, const uint8_t* mask,
                         const double* fib, const double* scale, double sig_l, double sig_t,
                         double h, double* tens /*6 arrays, scratch*/, double* c64[6],
                         float* c32[6]);

// two-level preconditioner of the bidomain inner solve (aggregates of
// bricks; see ep_kernels.hip): Kc = P^T K P into the zeroed dense kc (n x n,
// FP64) from the FP64 weights, K = c0 I + c1 A; kb: nb * kCoarseRow scratch,
// per brick its 27 neighbour-slot sums and (last) the sum of K's diagonal
constexpr int kCoarseRow = kNbr + 1;
void launch_coarse_setup(const LaunchCfg& L, const int* nbr, double* const ck64[6], double c0,
                         double c1, int n, const int* agg_ptr, const int* agg_brk, const int* agg,
                         double* kb, double* kc);
// kc += shift (every entry), then kc^-1 in place (blocked Gauss-Jordan,
// FP64, 32 columns per step); scratch: pinv 32 x 32, rp 32 x n, cp n x 32
// doubles
constexpr int kGjPanel = 32;
void launch_coarse_invert(hipStream_t st, int n, int ld, double* kc, double shift, double* pinv,
                          double* rp, double* cp);
// FP16 copy of kc * scale into kinv (n rows of ld entries, zero beyond n)
void launch_coarse_pack(hipStream_t st, int n, int ld, const double* kc, double scale,
                        void* kinv);
void launch_cg2_update(const LaunchCfg& L, float* x, float* r, float* p, float* s, const float* z,
                       const float* w, float* rb, int kind, const CGScalars* cin, CGScalars* cout,
                       const double* prev, unsigned long long* mirror, unsigned seq);
// cc = unscale * kinv (aggregate sums of rb), kinv the FP16 copy of
// launch_coarse_pack; with single-brick aggregates rb holds the sums already
// (rb and rc hold ld entries, zero beyond n)
void launch_coarse_apply(hipStream_t st, int n, int ld, bool brick_aggs, const int* agg_ptr,
                         const int* agg_brk, const float* rb, float* rc, const void* kinv,
                         float unscale, float* cc, const CGScalars* sc);
void launch_cg2_apply(const LaunchCfg& L, const int* nbr, CoefSet<float> c, float c0, float c1,
                      const float* dinv, const float* r, const float* cc, const int* agg, float* z,
                      float* w, const CGScalars* cin, double* parts);

// explicit step with A27 (ionic + diffusion + activation)
template <typename T>
void launch_explicit27(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* v,
                       const T* w, const T* jstim, T* vout, T* wout, T* tact, IonicT<T> ion,
                       T dt, T theta, double tn, int* flags);

// cross (nullable): records the step index where T_act is first set
template <typename T>
void launch_explicit(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* v,
                     const T* w, const T* jstim, T* vout, T* wout, T* tact,
                     IonicT<T> ion, T dt, T theta, double tn, int* flags, int* cross, int step);

// ---- several explicit steps per launch (ep_multistep.hip) -----------------
// Workgroups of the multi-step kernel that fit on the device at once (0: no
// cooperative launch); a grid with at most this many bricks can use it.
template <typename T>
int explicit_ms_capacity();
// nsteps explicit steps from step0 in one cooperative launch of nb
// workgroups (one brick each, one grid-wide barrier per step).  vin/win may
// alias vout/wout; xa, xb: (nb + 1) * 512 exchange arrays with a zero ghost
// brick; count: the barrier's arrival counter (cleared here, eagerly);
// flags[0]: non-finite potential, flags[2]: a barrier wait timed out.
template <typename T>
hipError_t launch_explicit_ms(hipStream_t st, int nb, const int* nbr, CoefSet<T> c,
                              const T* vin, const T* win, const T* jstim, T* vout, T* wout,
                              T* tact, T* xa, T* xb, IonicT<T> ion, T dt, T theta, double dt64,
                              long long step0, int nsteps, double* qacc, const double* qstep,
                              double qscale, unsigned* count, int* flags);

template <typename T>
void launch_ionic(const LaunchCfg& L, const T* v, const T* w, const T* jstim, T* vs,
                  T* wout, IonicT<T> ion, T dt);

// Persistent CG kernels (L.pgrid blocks).  Each launch reduces the partials
// `prev` of the launch before it (L.pgrid per component) into the solver
// scalars read from `cin`, publishes them in `cout` and leaves its own
// partials in `parts`.
//
// k_be_init: reaction, extrapolated x0, r0 = b - (I - dt A) x0, stored as
// z0 = M^-1 r0; optionally the activation check of the previous step (x
// still holds v_prev).  Partials (b.b, r.r).
template <typename T>
void launch_be_init(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* v,
                    const T* w, const T* jstim, const T* bprev, const T* qin, T kd,
                    const T* d2, const T* d3, T q2, T q3, T q4, T* bout, T* dout, T* qout,
                    T* x, T* wout, T* z, IonicT<T> ion, T dt, T* tact, T theta,
                    double tprev, int check_prev, int* flags, CGScalars* cout, double* parts,
                    double tol2, int maxit);


// One-launch-per-iteration PCG (textbook recurrences with the next
// residual norms expanded in the previous launch's dots; 7 partials per
// block), keeping z = M^-1 r and t = M^-1 q.  first: launch 0 of a solve
// (tests the init's (b.b, r.r)).
template <typename T>
void launch_pcg_step(const LaunchCfg& L, const int* nbr, CoefSet<T> c, T c0, T c1, T* x,
                     const T* z_in, T* z_out, const T* p_in, T* p_out, const T* t_in, T* t_out,
                     int first, const CGScalars* cin, CGScalars* cout, const double* prev,
                     double* parts, unsigned long long* mirror, unsigned seq);
constexpr int kMaxPartials = 7;   // partial sums per block of any CG launch

// field (brick layout, T) -> caller's device buffer in box layout (O);
// brick_id: box brick -> brick id or -1; fill for non-tissue voxels
template <typename T, typename O>
void launch_box_gather(hipStream_t s, const int n[3], int nby, int nbz, const int* brick_id,
                       const T* src, const uint8_t* mask, O* out, O fill);

// one Jacobi sweep x_out = x_in + M^-1 (b - (I - dt A) x_in) (L.grid blocks)
template <typename T>
void launch_jacobi(const LaunchCfg& L, const int* nbr, CoefSet<T> c, T dt, const T* dinv,
                   const T* b, const T* x_in, T* x_out);

// out[k] = sum of partials[k*nparts .. (k+1)*nparts) in a fixed order
void launch_reduce_sum(hipStream_t s, const double* partials, int nparts, int K, double* out);
void launch_block_max(const LaunchCfg& L, const int* nbr, CoefSet<double> c,
                      double* partials);
void launch_scale(const LaunchCfg& L, double* x, const double* y, const double* sums);

template <typename T>
void launch_activation(const LaunchCfg& L, const T* vold, const T* vnew, T* tact, T dt,
                       T theta, double tn, int* flags);

template <typename T>
void launch_dinv(const LaunchCfg& L, const int* nbr, CoefSet<T> c, T c0, T c1, T* dinv);

template <typename T>
void launch_sum(const LaunchCfg& L, const T* x, double* partials);

template <typename T>
void launch_stim_scatter(hipStream_t s, const int64_t* idx, const double* val, int n, T* jstim,
                         double* qstep);

void launch_q_accum(hipStream_t s, double* qacc, const double* qstep, double scale);

// bidomain
template <typename T>
void launch_resid64(const LaunchCfg& L, const int* nbr, CoefSet<double> ci, CoefSet<double> ck,
                    const T* vs, const double* phi, double* r64, double* partials);

void launch_inner_init(const LaunchCfg& L, const double* r64, const uint8_t* mask,
                       const double* sums, double inv_count, float* x, float* r,
                       CGScalars* cout, double* parts, double tol2, int maxit);

void launch_phi_correct(const LaunchCfg& L, double* phi, const float* d, const uint8_t* mask,
                        double* partials);

// phi = polynomial extrapolation (order 2 or 3) of the past solutions h1, h2, h3
void launch_phi_extrap(const LaunchCfg& L, double* phi, const double* h1, const double* h2,
                       const double* h3, int order);

void launch_phi_shift(const LaunchCfg& L, double* phi, const uint8_t* mask, const double* sum,
                      double inv_count);

template <typename T>
void launch_parabolic(const LaunchCfg& L, const int* nbr, CoefSet<T> ci, const T* vs,
                      const double* phi, const T* vold, T* vout, T* tact, T dt, T theta,
                      double tn, int* flags);

template <typename T>
void launch_apply(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* x, T* y,
                  double* partials);

// discrete adjoint of the explicit monodomain step (reverse mode)
template <typename T>
void launch_adj_init(const LaunchCfg& L, const uint8_t* mask, const T* vlast, const T* vprev,
                     const int* cross, const T* tact, const T* tstar, T* lv, T* lw, T dt,
                     T theta, int nlast);
template <typename T>
void launch_adj_step(const LaunchCfg& L, const int* nbr, CoefSet<T> c, CoefSet<T> d0,
                     const uint8_t* mask, const T* lv_in, const T* lw_in, T* lv_out, T* lw_out,
                     const T* v, const T* w, const T* jstim, const T* vnext, const T* vprev,
                     const int* cross, const T* tact, const T* tstar, double* grad,
                     IonicT<T> ion, T dt, T theta, T inv_h2, int n);
// unscaled voxel tensors D0 (6 component arrays) from unit fibres
template <typename T>
void launch_unit_tensors(const LaunchCfg& L, const uint8_t* mask, const double* fib,
                         double sig_l, double sig_t, T* out[6]);
template <typename T>
void launch_loss(const LaunchCfg& L, const uint8_t* mask, const int* cross, const T* tact,
                 const T* tstar, double* partials);

}  // namespace ep

// HIP kernels of the voxel-EP step for gfx950 (MI355X).
//
// One 512-thread workgroup (8 wavefronts) owns one 8x8x8 brick: thread t is
// voxel l = t (z fastest), so every wavefront touches one contiguous brick
// x-plane.  Stencil kernels stage the brick plus its face/edge halo (the
// 19-point operator needs no corner cells) in LDS, recomputing cheap
// pointwise work (the ionic update, the CG search direction) for halo cells
// instead of writing it to HBM and reading it back.  Every global load a
// thread needs (its own voxel, one halo cell, the 18 operator weights) is
// issued before the single barrier that publishes the tile, so the loads of
// a brick overlap instead of forming dependent round trips.  Nothing here is
// a dense contraction, so there is no MFMA: every kernel is HBM-bound.
//
// Reductions are deterministic and need no atomics: each block writes its
// FP64 partial sums to a fixed slot, and the next launch (every one of its
// blocks, redundantly) sums the previous launch's slots in a fixed order
// before using the totals.  The CG kernels are persistent (a fixed grid that
// strides over the bricks), so that sum costs a few hundred loads per block,
// and one CG iteration is one launch.  The FP32 implicit-step kernels also
// stage each block's next brick into LDS (direct global-to-LDS loads) while
// computing the current one, so the load wait of a brick overlaps the work
// of the one before it.
//
// What each kernel computes, with the passage it follows (thesis):
//   k_tensor, k_coefs, k_unit_tensor: voxel conductivity tensors (eqn:sigma1)
//     and the face / edge weights of the 19-point finite-volume operator
//     (matrix-free assembly, Linear Solver section, "Matrix-Free Assembly";
//     conductivity interpolated to the gradient points, Algorithm Details
//     chapter, Diffusion subsection).
//   k_explicit, k_ionic: Mitchell-Schaeffer reaction by explicit Euler
//     (eqn:ms1, eqn:ms2; Reaction subsection) fused with explicit diffusion;
//     activation time at the first threshold crossing.
//   k_be_init, k_pcg_step: implicit-Euler diffusion step (Linear Solver
//     section, "Implicit Euler") solved by Jacobi-preconditioned CG;
//     k_jacobi: the same step by the thesis's fixed Jacobi sweeps (eqn:iejac1);
//     k_cg2_update, k_coarse_gemv, k_cg2_apply (with k_coarse_brick and the
//     Gauss-Jordan set-up): the elliptic inner solve, one-reduction PCG with
//     a two-level (Jacobi + aggregate coarse space) preconditioner.
//   k_resid64, k_inner_init, k_phi_correct, k_phi_shift, k_parabolic: the
//     bidomain step (eqn:bidomain1): elliptic solve for phi_e by FP32 PCG
//     inside FP64 refinement, then the parabolic update.
//   k_adj_init, k_adj_step, k_loss: discrete adjoint of the explicit step
//     for the activation-time loss.
#include <cmath>

#include "ep_device.h"

namespace ep {
namespace {

using namespace dev;

// Brick m of this block in a persistent launch: XCD x = block % 8 owns the
// contiguous brick range [x*per, (x+1)*per); its blocks stride through it.
// Returns -1 when the block has no brick m.
__device__ __forceinline__ int pbrick(int m, int nb) {
  const int x = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
  const int gper = gridDim.x / kXcd;
  const int per = (nb + kXcd - 1) / kXcd;
  const int b = x * per + j + m * gper;
  return (b < (x + 1) * per && b < nb) ? b : -1;
}

// Neighbour row and row masks of a persistent block's next brick, loaded into
// registers of threads < 27 one brick ahead.  The loads for brick m+1 are
// issued as brick m starts and written to the other half of a double-buffered
// LDS table once brick m's own loads have landed (so no wait is added), before
// brick m's second barrier; brick m+1's data loads then follow its first
// barrier directly instead of waiting for a table load.
struct NbrAhead {
  int nbv = 0;
  uint64_t rmv = 0;
  __device__ __forceinline__ void fetch(const int* __restrict__ nbr,
                                        const uint64_t* __restrict__ rowsn, int brick) {
    // Unconditional and always in bounds (the tables hold at least the ghost
    // brick's row): a load under a branch would make the compiler wait for
    // every outstanding store before reissuing it.
    const int i = (brick < 0 ? 0 : brick) * kNbr + (threadIdx.x < kNbr ? threadIdx.x : 0);
    nbv = nbr[i];
    rmv = rowsn[i];
  }
  __device__ __forceinline__ void stage(int* nbs, uint64_t* rowm) const {
    if (threadIdx.x < kNbr) {
      nbs[threadIdx.x] = nbv;
      rowm[threadIdx.x] = rmv;
    }
  }
};

// Loads and stores of data no other brick of the launch reads (own-voxel
// streams, outputs).  With NT they carry the non-temporal hint, so that on
// grids whose working set exceeds the last-level cache they do not evict the
// halo and neighbour-weight lines the next bricks read; on grids that fit,
// plain accesses keep them cached for the next launch.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Sum the K partial sums the previous launch left (n per component) in a
// fixed order.  Every block computes the identical totals, so no block has
// to wait for another and nothing is communicated within the launch.
template <int K>
__device__ __forceinline__ void sum_prev(const double* __restrict__ parts, int n, double (&S)[K]) {
  __shared__ double red[K][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) x += parts[k * n + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[k][w];
    S[k] = t;
  }
  __syncthreads();
}

// A field in brick layout -> box layout (z fastest) in a caller's device
// buffer, converted to O; voxels that are not tissue get `fill`.
template <typename T, typename O>
__global__ __launch_bounds__(256) void k_box_gather(int n0, int n1, int n2, int nby, int nbz,
                                                    const int* __restrict__ brick_id,
                                                    const T* __restrict__ src,
                                                    const uint8_t* __restrict__ mask,
                                                    O* __restrict__ out, O fill) {
  const int64_t N = static_cast<int64_t>(n0) * n1 * n2;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += stride) {
    const int z = static_cast<int>(i % n2);
    const int64_t t = i / n2;
    const int y = static_cast<int>(t % n1), x = static_cast<int>(t / n1);
    const int b = brick_id[(static_cast<int64_t>(x >> 3) * nby + (y >> 3)) * nbz + (z >> 3)];
    O v = fill;
    if (b >= 0) {
      const int64_t g = static_cast<int64_t>(b) * kBV + (((x & 7) * 8 + (y & 7)) * 8 + (z & 7));
      if (mask[g]) v = static_cast<O>(src[g]);
    }
    out[i] = v;
  }
}

// ---------------------------------------------------------------------------
// coefficient encoding (once per conductivity change)
// ---------------------------------------------------------------------------
// Voxel tensors s (sT I + (sL - sT) f f^T) on the tissue (eqn:sigma1).  With
// body (the elliptic domain with a bath), voxels of the body outside the
// tissue get the isotropic bath tensor sig_body I: the extracellular / bath
// tensor field of the elliptic operator's second part.
__global__ __launch_bounds__(kBV) void k_tensor(int nb, const uint8_t* __restrict__ mask,
                                                const double* __restrict__ fib,
                                                const double* __restrict__ scale, double sig_l,
                                                double sig_t, double* __restrict__ tens,
                                                int64_t stride, const uint8_t* __restrict__ body,
                                                double sig_body) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  const bool t = mask[g] != 0;
  const double iso = (!t && body && body[g]) ? sig_body : 0.0;
  const double s = scale ? scale[g] : 1.0;
  const double f0 = fib[3 * (int64_t)g], f1 = fib[3 * (int64_t)g + 1], f2 = fib[3 * (int64_t)g + 2];
  const double a = sig_l - sig_t;
  tens[0 * stride + g] = t ? s * (sig_t + a * f0 * f0) : iso;
  tens[1 * stride + g] = t ? s * (sig_t + a * f1 * f1) : iso;
  tens[2 * stride + g] = t ? s * (sig_t + a * f2 * f2) : iso;
  tens[3 * stride + g] = t ? s * (a * f0 * f1) : 0.0;
  tens[4 * stride + g] = t ? s * (a * f0 * f2) : 0.0;
  tens[5 * stride + g] = t ? s * (a * f1 * f2) : 0.0;
}

// unscaled voxel tensors (scale 1) in state precision, 6 component arrays
template <typename T>
__global__ __launch_bounds__(kBV) void k_unit_tensor(int nb, const uint8_t* __restrict__ mask,
                                                     const double* __restrict__ fib, double sig_l,
                                                     double sig_t, CoefOut<T> out) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  const bool t = mask[g] != 0;
  const double f0 = fib[3 * (int64_t)g], f1 = fib[3 * (int64_t)g + 1], f2 = fib[3 * (int64_t)g + 2];
  const double a = sig_l - sig_t;
  const double d[6] = {sig_t + a * f0 * f0, sig_t + a * f1 * f1, sig_t + a * f2 * f2,
                       a * f0 * f1,         a * f0 * f2,         a * f1 * f2};
#pragma unroll
  for (int k = 0; k < 6; ++k) out.c[k][g] = t ? static_cast<T>(d[k]) : T(0);
}

// Face weight: mean of the two voxel tensors / h^2 when both are tissue.
// Edge weight: mean of the four voxel tensors of the 2x2 block / (2 h^2)
// when all four are tissue.  Terms touching non-tissue are dropped (no flux).
__global__ __launch_bounds__(kBV) void k_coefs(int nb, const int* __restrict__ nbr,
                                               const uint8_t* __restrict__ mask,
                                               const double* __restrict__ tens, int64_t stride,
                                               double inv_h2, CoefOut<double> out64,
                                               CoefOut<float> out32) {
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  const int t = threadIdx.x;
  if (t < kNbr) nbs[t] = nbr[brick * kNbr + t];
  __syncthreads();
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  const int g = brick * kBV + t;
  const int gx = nb_global(nbs, brick, lx, ly, lz, 1, 0, 0);
  const int gy = nb_global(nbs, brick, lx, ly, lz, 0, 1, 0);
  const int gz = nb_global(nbs, brick, lx, ly, lz, 0, 0, 1);
  const int gxy = nb_global(nbs, brick, lx, ly, lz, 1, 1, 0);
  const int gxz = nb_global(nbs, brick, lx, ly, lz, 1, 0, 1);
  const int gyz = nb_global(nbs, brick, lx, ly, lz, 0, 1, 1);
  const bool m0 = mask[g] != 0, mx = mask[gx] != 0, my = mask[gy] != 0, mz = mask[gz] != 0;
  const bool mxy = mask[gxy] != 0, mxz = mask[gxz] != 0, myz = mask[gyz] != 0;
  double c[6];
  c[CX] = (m0 && mx) ? 0.5 * (tens[0 * stride + g] + tens[0 * stride + gx]) * inv_h2 : 0.0;
  c[CY] = (m0 && my) ? 0.5 * (tens[1 * stride + g] + tens[1 * stride + gy]) * inv_h2 : 0.0;
  c[CZ] = (m0 && mz) ? 0.5 * (tens[2 * stride + g] + tens[2 * stride + gz]) * inv_h2 : 0.0;
  c[CXY] = (m0 && mx && my && mxy)
               ? 0.25 * (tens[3 * stride + g] + tens[3 * stride + gx] + tens[3 * stride + gy] +
                         tens[3 * stride + gxy]) * (0.5 * inv_h2)
               : 0.0;
  c[CXZ] = (m0 && mx && mz && mxz)
               ? 0.25 * (tens[4 * stride + g] + tens[4 * stride + gx] + tens[4 * stride + gz] +
                         tens[4 * stride + gxz]) * (0.5 * inv_h2)
               : 0.0;
  c[CYZ] = (m0 && my && mz && myz)
               ? 0.25 * (tens[5 * stride + g] + tens[5 * stride + gy] + tens[5 * stride + gz] +
                         tens[5 * stride + gyz]) * (0.5 * inv_h2)
               : 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (out64.c[k]) out64.c[k][g] = c[k];
    if (out32.c[k]) out32.c[k][g] = static_cast<float>(c[k]);
  }
}

// acc += add, weight by weight, with an FP32 copy of the sum.  The bidomain
// elliptic operator is the sum of the intracellular operator on the heart
// and the extracellular (and bath) operator over the elliptic domain, each
// assembled over its own domain (eqn:bidomain1 with its boundary
// conditions).
__global__ __launch_bounds__(kBV) void k_coef_add(int nb, CoefOut<double> acc,
                                                  CoefSet<double> add, CoefOut<float> out32) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double s = acc.c[k][g] + add.c[k][g];
    acc.c[k][g] = s;
    out32.c[k][g] = static_cast<float>(s);
  }
}

// Corner tensors of the corner-gradient operator A27 (Matrix-Free Assembly
// section with the conductivity block of the Diffusion subsection).  Voxel p
// owns the corner at p + (1/2, 1/2, 1/2) h, where the 2x2x2 block p + {0,1}^3
// meets.  Its six tensor entries (xx, yy, zz, xy, xz, yz) are the mean of the
// block's eight voxel tensors over 16 h^2, or zero when the block holds a
// non-tissue voxel (no flux through that corner).  With these weights
//   (A27 v)_p = sum over p's 8 corners c of sigma_c . (K_c u_c),
// sigma_c the sign vector of c - p and u_c the block's signed sums
// (sum over the block of sign(q - c)_d v_q for each axis d).
__global__ __launch_bounds__(kBV) void k_coefs27(int nb, const int* __restrict__ nbr,
                                                 const uint8_t* __restrict__ mask,
                                                 const double* __restrict__ tens, int64_t stride,
                                                 double inv_16h2, CoefOut<double> out64,
                                                 CoefOut<float> out32) {
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  const int t = threadIdx.x;
  if (t < kNbr) nbs[t] = nbr[brick * kNbr + t];
  __syncthreads();
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  int gq[8];
  bool full = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    gq[k] = nb_global(nbs, brick, lx, ly, lz, k >> 2, (k >> 1) & 1, k & 1);
    full = full && mask[gq[k]] != 0;
  }
  const int g = brick * kBV + t;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) a += tens[m * stride + gq[k]];
    const double cval = full ? a * 0.125 * inv_16h2 : 0.0;
    if (out64.c[m]) out64.c[m][g] = cval;
    if (out32.c[m]) out32.c[m][g] = static_cast<float>(cval);
  }
}

// ---------------------------------------------------------------------------
// explicit monodomain step: ionic + 19-point diffusion + activation, fused
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBV) void k_explicit(int nb, const int* __restrict__ nbr,
                                                  CoefSet<T> c, const T* __restrict__ v,
                                                  const T* __restrict__ w,
                                                  const T* __restrict__ jstim,
                                                  T* __restrict__ vout, T* __restrict__ wout,
                                                  T* __restrict__ tact, IonicT<T> ion, T dt,
                                                  T theta, double tn, int* flags,
                                                  int* __restrict__ cross, int step) {
  __shared__ T s[kTile];
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  const T v0 = at(v, q.g), w0 = at(w, q.g);
  const T j0 = jstim ? at(jstim, q.g) : T(0);
  T hv = T(0), hw = T(0), hj = T(0);
  if (q.has_halo) {
    hv = at(v, q.hg);
    hw = at(w, q.hg);
    hj = jstim ? at(jstim, q.hg) : T(0);
  }
  T k18[18];
  gather18(c, nbs, brick, q.lx, q.ly, q.lz, k18);
  T vs, ws;
  ms_step(v0, w0, j0, ion, dt, vs, ws);
  s[q.C] = vs;
  if (q.has_halo) {
    T a, b;
    ms_step(hv, hw, hj, ion, dt, a, b);
    s[q.hC] = a;
  }
  __syncthreads();
  const T vn = vs + dt * apply19(s, q.C, k18);
  at(vout, q.g) = vn;
  at(wout, q.g) = ws;
  if (v0 < theta && theta <= vn) {
    if (isinf(at(tact, q.g))) {
      at(tact, q.g) = static_cast<T>(tn) + dt * (theta - v0) / (vn - v0);
      if (cross) at(cross, q.g) = step;
    }
  }
  if (!isfinite(vn)) flags[0] = 1;
}

// ---------------------------------------------------------------------------
// explicit monodomain step with the corner-gradient operator A27: ionic +
// diffusion + activation, fused.  Two phases over the brick's LDS tile:
// every corner of the brick's voxels (9^3 of them, lower voxel at tile
// coordinates [0, 8]^3) gets its flux K_c u_c once, then each voxel sums the
// signed fluxes of its 8 corners.  Thread t takes the corner its own voxel
// owns (tile coordinates in [1, 8]^3, so its six weights are plain
// coalesced loads), and threads < 217 also take one corner owned by the
// -x / -y / -z halo (a tile coordinate of 0).
// ---------------------------------------------------------------------------
constexpr int kCorners = 729;            // 9^3 corners per brick
constexpr int kCornersExtra = 729 - 512; // corners with a tile coordinate of 0

__device__ __forceinline__ int corner_id(int cx, int cy, int cz) { return (cx * 9 + cy) * 9 + cz; }

// the k-th corner (k < 217) with a lower-voxel tile coordinate equal to 0
__device__ __forceinline__ void extra_corner(int k, int& cx, int& cy, int& cz) {
  if (k < 81) { cx = 0; cy = k / 9; cz = k % 9; }
  else if (k < 153) { k -= 81; cx = (k / 9) + 1; cy = 0; cz = k % 9; }
  else { k -= 153; cx = (k >> 3) + 1; cy = (k & 7) + 1; cz = 0; }
}

template <typename T>
__device__ __forceinline__ void corner_flux(const T* s, int cx, int cy, int cz, const T k[6],
                                            T* qx, T* qy, T* qz) {
  const int b = tidx(cx, cy, cz);
  // block values v[i][j][l] at tile (cx+i, cy+j, cz+l)
  const T v000 = s[b], v001 = s[b + 1], v010 = s[b + 10], v011 = s[b + 11];
  const T v100 = s[b + 100], v101 = s[b + 101], v110 = s[b + 110], v111 = s[b + 111];
  const T ux = (v100 - v000) + (v101 - v001) + (v110 - v010) + (v111 - v011);
  const T uy = (v010 - v000) + (v011 - v001) + (v110 - v100) + (v111 - v101);
  const T uz = (v001 - v000) + (v011 - v010) + (v101 - v100) + (v111 - v110);
  const int ci = corner_id(cx, cy, cz);
  qx[ci] = k[CX] * ux + k[CXY] * uy + k[CXZ] * uz;
  qy[ci] = k[CXY] * ux + k[CY] * uy + k[CYZ] * uz;
  qz[ci] = k[CXZ] * ux + k[CYZ] * uy + k[CZ] * uz;
}

template <typename T>
__global__ __launch_bounds__(kBV) void k_explicit27(int nb, const int* __restrict__ nbr,
                                                    CoefSet<T> c, const T* __restrict__ v,
                                                    const T* __restrict__ w,
                                                    const T* __restrict__ jstim,
                                                    T* __restrict__ vout, T* __restrict__ wout,
                                                    T* __restrict__ tact, IonicT<T> ion, T dt,
                                                    T theta, double tn, int* flags) {
  __shared__ T s[kTile];
  __shared__ T qx[kCorners], qy[kCorners], qz[kCorners];
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  const T v0 = at(v, q.g), w0 = at(w, q.g);
  const T j0 = jstim ? at(jstim, q.g) : T(0);
  T hv = T(0), hw = T(0), hj = T(0);
  if (q.has_halo) {
    hv = at(v, q.hg);
    hw = at(w, q.hg);
    hj = jstim ? at(jstim, q.hg) : T(0);
  }
  // the 8 corner cells of the tile, which the 19-point halo leaves out
  const bool tcorner = threadIdx.x >= kHalo && threadIdx.x < kHalo + 8;
  int cC = 0;
  T cv = T(0), cw = T(0), cj = T(0);
  if (tcorner) {
    const int k = threadIdx.x - kHalo;
    const int hx = (k & 4) ? 9 : 0, hy = (k & 2) ? 9 : 0, hz = (k & 1) ? 9 : 0;
    const int cg = tile_global(nbs, hx, hy, hz);
    cC = tidx(hx, hy, hz);
    cv = v[cg];
    cw = w[cg];
    cj = jstim ? jstim[cg] : T(0);
  }
  // this thread's corners: the one its own voxel owns, and for threads < 217
  // one with a tile coordinate of 0
  T k1[6], k2[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) k1[m] = c.c[m][q.g];
  const bool two = threadIdx.x < kCornersExtra;
  int cx2 = 0, cy2 = 0, cz2 = 0;
  if (two) {
    extra_corner(threadIdx.x, cx2, cy2, cz2);
    const int g2 = nb_global(nbs, brick, cx2 - 1, cy2 - 1, cz2 - 1, 0, 0, 0);
#pragma unroll
    for (int m = 0; m < 6; ++m) k2[m] = c.c[m][g2];
  }
  T vs, ws;
  ms_step(v0, w0, j0, ion, dt, vs, ws);
  s[q.C] = vs;
  if (q.has_halo) {
    T a, b;
    ms_step(hv, hw, hj, ion, dt, a, b);
    s[q.hC] = a;
  }
  if (tcorner) {
    T a, b;
    ms_step(cv, cw, cj, ion, dt, a, b);
    s[cC] = a;
  }
  __syncthreads();
  corner_flux(s, q.lx + 1, q.ly + 1, q.lz + 1, k1, qx, qy, qz);
  if (two) corner_flux(s, cx2, cy2, cz2, k2, qx, qy, qz);
  __syncthreads();
  T a = T(0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        const int ci = corner_id(q.lx + i, q.ly + j, q.lz + l);
        const T fx = i ? qx[ci] : -qx[ci];
        const T fy = j ? qy[ci] : -qy[ci];
        const T fz = l ? qz[ci] : -qz[ci];
        a += fx + fy + fz;
      }
  const T vn = vs + dt * a;
  at(vout, q.g) = vn;
  at(wout, q.g) = ws;
  if (v0 < theta && theta <= vn && isinf(at(tact, q.g)))
    at(tact, q.g) = static_cast<T>(tn) + dt * (theta - v0) / (vn - v0);
  if (!isfinite(vn)) flags[0] = 1;
}

// pointwise ionic update (bidomain reaction sub-step)
template <typename T>
__global__ __launch_bounds__(kBV) void k_ionic(int nb, const T* __restrict__ v,
                                               const T* __restrict__ w,
                                               const T* __restrict__ jstim, T* __restrict__ vs,
                                               T* __restrict__ wout, IonicT<T> ion, T dt) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  T a, b;
  ms_step(v[g], w[g], jstim ? jstim[g] : T(0), ion, dt, a, b);
  vs[g] = a;
  wout[g] = b;
}

// ---------------------------------------------------------------------------
// implicit Euler diffusion by Jacobi-PCG:  (I - dt A) x = v*,  x0 = v*
// ---------------------------------------------------------------------------
// The CG kernels run persistently (about four blocks per CU, each looping
// over its bricks).  Each launch first sums the partial sums the previous
// launch left (one per block, fixed order, identical in every block), updates
// the solver scalars from them, and block 0 publishes the scalars for the
// host and the next launch.  Partials and scalars are double-buffered: a
// launch reads `prev` / `cin` and writes `parts` / `cout`.
//
// The elliptic inner solve uses the one-reduction form of preconditioned CG
// (Chronopoulos and Gear): with u = M^-1 r and w = K u it carries s = K p by
// recurrence,
//   gamma = (r, u), delta = (u, w),  beta = gamma / gamma_old,
//   alpha = gamma / (delta - beta gamma / alpha_old),
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
// so its three dot products share one reduction.

// ---------------------------------------------------------------------------
// Pipelined brick loop of the FP32 implicit-step kernels (the CG launches
// and the init kernel below).  A block's next brick is staged into LDS by
// direct global-to-LDS loads while the current brick is computed, so its
// load latency overlaps that work instead of following it.  For the CG
// launches a stage holds:
//   own cells of z, t, p, x and of the six weight arrays (lane order = the
//   brick's voxel order), the 480 halo cells of z and t (halo_cell order),
//   and the 600 weights of cells on the brick's -x, -y, -z sides that the
//   19-point operator of its own voxels uses (the weight halo, below).
// Every staged value is the one gather18 / cell_setup would load (rows
// without tissue read the ghost brick's zeros), and the arithmetic is the
// one-brick-at-a-time loop's, so the results are bitwise those of that
// loop.  A brick's outputs are stored one stage later, after the
// next staging loads are issued, so that the wait for a stage does not also
// wait for the stores just issued.
// A stage is one flat LDS array, so that every access to it has the same
// underlying object and the compiler can tell the stage being read from the
// one being filled.  (The weight halo and the staging helpers are in
// ep_device.h.)
constexpr int kStZ = 0, kStT = 512, kStP = 1024, kStX = 1536, kStW = 2048;   // own cells
constexpr int kStHZ = 5120, kStHT = 5632;                                    // halo cells
constexpr int kStWH = 6144;                                                  // weight halo
constexpr int kStage = kStWH + kWHalo;

// issue the staging loads of `brick` (table nbs / rowm in LDS) into F; the
// first launch of a solve reads z alone (t, p, x are not yet formed)
template <bool NT, bool FIRST>
__device__ __forceinline__ void pcg_stage(float* F, int brick, int nb, const int* nbs,
                                          const uint64_t* rowm, const CoefSet<float>& c,
                                          const float* x, const float* z_in, const float* p_in,
                                          const float* t_in) {
  const int t = threadIdx.x, w0 = t & ~63;
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  const int gl = vox_live(rowm, lx, ly, lz) ? brick * kBV + t : nb * kBV + t;
  lds_load<false>(z_in, gl, F + kStZ + w0);
  if constexpr (!FIRST) {
    lds_load<false>(t_in, gl, F + kStT + w0);
    lds_load<false>(p_in, gl, F + kStP + w0);
    lds_load<NT>(x, gl, F + kStX + w0);
  }
  if (t < kHalo) {
    const int hgl = halo_index(t, nb, nbs, rowm);
    lds_load<false>(z_in, hgl, F + kStHZ + w0);
    if constexpr (!FIRST) lds_load<false>(t_in, hgl, F + kStHT + w0);
  }
  stage_weights<kStW, kStWH>(F, gl, nb, nbs, rowm, c);
}

// The CG launches' brick loop, pipelined (see pcg_stage): alpha, beta from
// this launch's scalars; partials as the one-brick-at-a-time loop.  FIRST:
// launch 0 (t, p, x taken as zero, only p and t stored).
// S0, S1: the two stages (kStage floats each); s: the tile; nbt, rowt: the
// double-buffered neighbour table and row masks (2 x kNbr each).
template <bool NT, bool FIRST>
__device__ __forceinline__ void pcg_iter_pipelined(
    float* S0, float* S1, float* s, int (*nbt)[kNbr], uint64_t (*rowt)[kNbr], int nb,
    const int* __restrict__ nbr, const uint64_t* __restrict__ rowsn,
    const CoefSet<float>& c, float c0, float c1, float alpha, float beta,
    float* __restrict__ x, const float* __restrict__ z_in, float* __restrict__ z_out,
    const float* __restrict__ p_in, float* __restrict__ p_out, const float* __restrict__ t_in,
    float* __restrict__ t_out, double* parts) {
  const int t = threadIdx.x;
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  const int C = tidx(lx + 1, ly + 1, lz + 1);
  int hC = 0;
  if (t < kHalo) {
    int hx, hy, hz;
    halo_cell(t, hx, hy, hz);
    hC = tidx(hx, hy, hz);
  }
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  NbrAhead ahead;
  // outputs of the previous brick, stored one stage later
  int pend_brick = -1;   // the same in every thread
  bool pend = false;
  float ox = 0.f, oz = 0.f, op = 0.f, ot = 0.f;
  int cur = pbrick(0, nb);
  ahead.fetch(nbr, rowsn, cur);
  ahead.stage(nbt[0], rowt[0]);
  __syncthreads();
  if (cur >= 0) pcg_stage<NT, FIRST>(S0, cur, nb, nbt[0], rowt[0], c, x, z_in, p_in, t_in);
  ahead.fetch(nbr, rowsn, pbrick(1, nb));
  // one brick: S holds its stage, N receives the next brick's
  auto brick_step = [&](const float* S, float* N, int m) -> bool {
    if (cur < 0) return false;
    __builtin_amdgcn_s_waitcnt(0);   // this wave's staging loads have landed
    __syncthreads();                 // every wave's; the previous brick is done with LDS
    const bool live = vox_live(rowt[m & 1], lx, ly, lz);
    const float tg = FIRST ? 0.f : S[kStT + t];
    const float zn = S[kStZ + t] - alpha * tg;
    s[C] = zn;
    if (t < kHalo) s[hC] = S[kStHZ + t] - alpha * (FIRST ? 0.f : S[kStHT + t]);
    ahead.stage(nbt[(m + 1) & 1], rowt[(m + 1) & 1]);
    __syncthreads();
    const int nxt = pbrick(m + 1, nb);
    if (nxt >= 0)
      pcg_stage<NT, FIRST>(N, nxt, nb, nbt[(m + 1) & 1], rowt[(m + 1) & 1], c, x, z_in, p_in,
                           t_in);
    ahead.fetch(nbr, rowsn, pbrick(m + 2, nb));
    if (pend) {
      const int g = pend_brick * kBV + t;
      if constexpr (!FIRST) {
        st_stream<NT>(&at(x, g), ox);
        st_stream<NT>(&at(z_out, g), oz);
      }
      st_stream<NT>(&at(p_out, g), op);
      st_stream<NT>(&at(t_out, g), ot);
    }
    float k18[18];
    gather18_lds<kStW, kStWH>(S, t, lx, ly, lz, k18);
    if (!live) {
#pragma unroll
      for (int i = 0; i < 18; ++i) k18[i] = 0.f;
    }
    const float pg = FIRST ? 0.f : S[kStP + t], xg = FIRST ? 0.f : S[kStX + t];
    // q_k = K p_k = K z_k + beta q_{k-1}, with q_{k-1} = M t_{k-1}
    const float md = c0 + c1 * diag19(k18);
    const float qn = (c0 * zn + c1 * apply19(s, C, k18)) + beta * (md * tg);
    const float pn = zn + beta * pg;
    const float tn = qn / md;
    const float rn = md * zn;
    pend = live;
    pend_brick = cur;
    ox = xg + alpha * pg;
    oz = zn;
    op = pn;
    ot = tn;
    const double dr = rn, dz = zn, dp = pn, dq = qn;
    acc[0] += dp * dq;
    acc[1] += dr * dz;
    acc[2] += dq * dz;
    acc[3] += dq * static_cast<double>(tn);
    acc[4] += dr * dr;
    acc[5] += dq * dr;
    acc[6] += dq * dq;
    cur = nxt;
    return true;
  };
  for (int m = 0;; m += 2) {
    if (!brick_step(S0, S1, m)) break;
    if (!brick_step(S1, S0, m + 1)) break;
  }
  if (pend) {
    const int g = pend_brick * kBV + t;
    if constexpr (!FIRST) {
      st_stream<NT>(&at(x, g), ox);
      st_stream<NT>(&at(z_out, g), oz);
    }
    st_stream<NT>(&at(p_out, g), op);
    st_stream<NT>(&at(t_out, g), ot);
  }
  block_partials<7>(acc, parts);
}

// Stage of the pipelined init kernel (flat, floats): own cells of v, w, the
// previous v, b_{n-1}, Q_n, d_{n-2}, d_{n-3} and the six weights, halo cells
// (480 each) of v, w, b_{n-1}, Q_n, then the weight halo.  The stimulus
// current, present only while a stimulus is on, is read directly.
constexpr int kIV = 0, kIW = 512, kIVP = 1024, kIB1 = 1536, kIQ0 = 2048, kID2 = 2560,
              kID3 = 3072, kIWt = 3584;
constexpr int kIHV = 6656, kIHW = kIHV + kHalo, kIHB = kIHW + kHalo, kIHQ = kIHB + kHalo;
constexpr int kIWH = kIHQ + kHalo;
constexpr int kIStage = kIWH + kWHalo;

struct BeInitArgs {
  const float *v, *w, *jstim, *bprev, *qin, *d2in, *d3in;
  float *bout, *dout, *qout, *x, *wout, *z;
  float kd, q2, q3, q4;
  bool check_prev;
};

template <bool NT>
__device__ __forceinline__ void be_init_stage(float* F, int brick, int nb, const int* nbs,
                                              const uint64_t* rowm, const CoefSet<float>& c,
                                              const BeInitArgs& A) {
  const int t = threadIdx.x, w0 = t & ~63;
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  const int gl = vox_live(rowm, lx, ly, lz) ? brick * kBV + t : nb * kBV + t;
  lds_load<false>(A.v, gl, F + kIV + w0);
  lds_load<false>(A.w, gl, F + kIW + w0);
  if (A.check_prev) lds_load<NT>(A.x, gl, F + kIVP + w0);
  if (A.bprev) lds_load<false>(A.bprev, gl, F + kIB1 + w0);
  if (A.qin) lds_load<false>(A.qin, gl, F + kIQ0 + w0);
  if (A.d2in) lds_load<NT>(A.d2in, gl, F + kID2 + w0);
  if (A.d3in) lds_load<NT>(A.d3in, gl, F + kID3 + w0);
  if (t < kHalo) {
    const int hgl = halo_index(t, nb, nbs, rowm);
    lds_load<false>(A.v, hgl, F + kIHV + w0);
    lds_load<false>(A.w, hgl, F + kIHW + w0);
    if (A.bprev) lds_load<false>(A.bprev, hgl, F + kIHB + w0);
    if (A.qin) lds_load<false>(A.qin, hgl, F + kIHQ + w0);
  }
  stage_weights<kIWt, kIWH>(F, gl, nb, nbs, rowm, c);
}

// k_be_init's brick loop, pipelined like the CG launches (see pcg_stage);
// the arithmetic is the one-brick-at-a-time loop's, so the results are
// bitwise the same.
template <bool NT>
__device__ __forceinline__ void be_init_pipelined(
    float* S0, float* S1, float* s, int (*nbt)[kNbr], uint64_t (*rowt)[kNbr], int nb,
    const int* __restrict__ nbr, const uint64_t* __restrict__ rowsn, const CoefSet<float>& c,
    const BeInitArgs& A, const IonicT<float>& ion, float dt, float* __restrict__ tact,
    float theta, double tprev, int* flags, double* parts) {
  const int t = threadIdx.x;
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  const int C = tidx(lx + 1, ly + 1, lz + 1);
  int hC = 0;
  if (t < kHalo) {
    int hx, hy, hz;
    halo_cell(t, hx, hy, hz);
    hC = tidx(hx, hy, hz);
  }
  double acc[2] = {0.0, 0.0};
  NbrAhead ahead;
  int pend_brick = -1;   // the same in every thread
  bool pend = false;
  float o_x = 0.f, o_b = 0.f, o_d = 0.f, o_q = 0.f, o_w = 0.f, o_z = 0.f;
  int cur = pbrick(0, nb);
  ahead.fetch(nbr, rowsn, cur);
  ahead.stage(nbt[0], rowt[0]);
  __syncthreads();
  if (cur >= 0) be_init_stage<NT>(S0, cur, nb, nbt[0], rowt[0], c, A);
  ahead.fetch(nbr, rowsn, pbrick(1, nb));
  auto flush = [&]() {
    if (!pend) return;
    const int g = pend_brick * kBV + t;
    st_stream<NT>(&at(A.x, g), o_x);
    st_stream<NT>(&at(A.bout, g), o_b);
    if (A.bprev) {
      st_stream<NT>(&at(A.dout, g), o_d);
      st_stream<NT>(&at(A.qout, g), o_q);
    }
    st_stream<NT>(&at(A.wout, g), o_w);
    st_stream<NT>(&at(A.z, g), o_z);
  };
  auto brick_step = [&](const float* S, float* N, int m) -> bool {
    if (cur < 0) return false;
    __builtin_amdgcn_s_waitcnt(0);   // this wave's staging loads have landed
    __syncthreads();                 // every wave's; the previous brick is done with LDS
    const uint64_t* rowm = rowt[m & 1];
    const int* nbs = nbt[m & 1];
    const bool live = vox_live(rowm, lx, ly, lz);
    const int gl = live ? cur * kBV + t : nb * kBV + t;
    const float v0 = S[kIV + t], w0 = S[kIW + t];
    const float j0 = A.jstim ? at(A.jstim, gl) : 0.f;
    const float b1 = A.bprev ? S[kIB1 + t] : 0.f;
    const float q0 = A.qin ? S[kIQ0 + t] : 0.f;
    float vs, ws;
    ms_step(v0, w0, j0, ion, dt, vs, ws);
    const float d1 = v0 - b1;
    const float x0 = A.bprev ? vs + (A.kd * d1 + q0) : vs;
    s[C] = x0;
    if (t < kHalo) {
      const float hv = S[kIHV + t], hw = S[kIHW + t];
      const float hj = A.jstim ? at(A.jstim, halo_index(t, nb, nbs, rowm)) : 0.f;
      const float hb1 = A.bprev ? S[kIHB + t] : 0.f;
      const float hq = A.qin ? S[kIHQ + t] : 0.f;
      float a, b;
      ms_step(hv, hw, hj, ion, dt, a, b);
      s[hC] = A.bprev ? a + (A.kd * (hv - hb1) + hq) : a;
    }
    ahead.stage(nbt[(m + 1) & 1], rowt[(m + 1) & 1]);
    __syncthreads();
    const int nxt = pbrick(m + 1, nb);
    if (nxt >= 0) be_init_stage<NT>(N, nxt, nb, nbt[(m + 1) & 1], rowt[(m + 1) & 1], c, A);
    ahead.fetch(nbr, rowsn, pbrick(m + 2, nb));
    flush();
    float k18[18];
    gather18_lds<kIWt, kIWH>(S, t, lx, ly, lz, k18);
    if (!live) {
#pragma unroll
      for (int i = 0; i < 18; ++i) k18[i] = 0.f;
    }
    const float rr = (vs - x0) + dt * apply19(s, C, k18);
    // z0 = M^-1 r0, M the diagonal of I - dt A from this voxel's weights
    const float z0 = rr / (1.f - dt * diag19(k18));
    const float vp = A.check_prev ? S[kIVP + t] : 0.f;
    if (A.check_prev && vp < theta && theta <= v0) {
      const int g = cur * kBV + t;
      if (isinf(at(tact, g))) at(tact, g) = static_cast<float>(tprev) + dt * (theta - vp) / (v0 - vp);
    }
    if (!isfinite(v0)) flags[0] = 1;
    pend = live;
    pend_brick = cur;
    o_x = x0;
    o_b = vs;
    o_d = d1;
    o_q = A.q2 * d1 + A.q3 * (A.d2in ? S[kID2 + t] : 0.f) + A.q4 * (A.d3in ? S[kID3 + t] : 0.f);
    o_w = ws;
    o_z = z0;
    const double rd = static_cast<double>(rr);
    acc[0] += static_cast<double>(vs) * static_cast<double>(vs);
    acc[1] += rd * rd;
    cur = nxt;
    return true;
  };
  for (int m = 0;; m += 2) {
    if (!brick_step(S0, S1, m)) break;
    if (!brick_step(S1, S0, m + 1)) break;
  }
  flush();
  block_partials<2>(acc, parts);
}

// Reaction fused with the initial guess and residual of the implicit solve
// (I - dt A) x = b, b = v*.  The guess extrapolates the diffusion increment
// d_k = v_{k+1} - b_k of the past steps by the polynomial through the last
// K <= 4 of them (binomial weights): x0 = b + K d_{n-1} + Q_n, where
// d_{n-1} = v_n - b_{n-1} (bprev) and Q_n, the part that holds only older
// increments, was stored by the previous step (qin; none for K <= 1).  This
// step stores b (bout), d_{n-1} (dout) and
//   Q_{n+1} = q2 d_{n-1} + q3 d_{n-2} + q4 d_{n-3}   (qout; d2, d3 older ones)
// for the next one.  No buffer read here is written in the same launch, so
// halo reads never race with other blocks' writes.  r0 = b - (I - dt A) x0;
// the solve keeps z0 = M^-1 r0 (M the diagonal of I - dt A).
// When check_prev is set it also records activation for the previous step
// (vprev -> v) before x0 overwrites vprev's buffer.
// Partials: (b.b, r.r).  FP32 grids run the pipelined overload below.
template <typename T, bool NT>
__global__ __launch_bounds__(kBV) void k_be_init(int nb, const int* __restrict__ nbr,
                                                 CoefSet<T> c, const T* __restrict__ v,
                                                 const T* __restrict__ w,
                                                 const T* __restrict__ jstim,
                                                 const T* __restrict__ bprev,
                                                 const T* __restrict__ qin, T kd,
                                                 const T* __restrict__ d2in,
                                                 const T* __restrict__ d3in, T q2, T q3, T q4,
                                                 T* __restrict__ bout, T* __restrict__ dout,
                                                 T* __restrict__ qout, T* x,
                                                 T* __restrict__ wout, T* __restrict__ z,
                                                 IonicT<T> ion, T dt, T* __restrict__ tact,
                                                 T theta, double tprev, int check_prev,
                                                 int* flags, CGScalars* cout, double* parts,
                                                 double tol2, int maxit,
                                                 const uint64_t* __restrict__ rowsn) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CGScalars st = {};
    st.tol2 = tol2;
    st.maxit = maxit;
    *cout = st;
  }
  __shared__ T s[kTile];
  __shared__ int nbt[2][kNbr];
  __shared__ uint64_t rowt[2][kNbr];
  double acc[2] = {0.0, 0.0};
  NbrAhead ahead;
  int nxt = pbrick(0, nb);
  ahead.fetch(nbr, rowsn, nxt);
  ahead.stage(nbt[0], rowt[0]);
  for (int m = 0; nxt >= 0; ++m) {
    const int brick = nxt;
    const int* nbs = nbt[m & 1];
    const uint64_t* rowm = rowt[m & 1];
    nxt = pbrick(m + 1, nb);
    ahead.fetch(nbr, rowsn, nxt);
    __syncthreads();
    const Cell q = cell_setup(nbs, brick, rowm, nb);
    const T v0 = at(v, q.gl), w0 = at(w, q.gl);
    const T j0 = jstim ? at(jstim, q.gl) : T(0);
    const T vp = check_prev ? ld_stream<NT>(&at(x, q.gl)) : T(0);
    const T b1 = bprev ? at(bprev, q.gl) : T(0);
    const T q0 = qin ? at(qin, q.gl) : T(0);
    const T d2 = d2in ? ld_stream<NT>(&at(d2in, q.gl)) : T(0);
    const T d3 = d3in ? ld_stream<NT>(&at(d3in, q.gl)) : T(0);
    T hv = T(0), hw = T(0), hj = T(0), hb1 = T(0), hq = T(0);
    if (q.has_halo) {
      hv = at(v, q.hgl);
      hw = at(w, q.hgl);
      hj = jstim ? at(jstim, q.hgl) : T(0);
      hb1 = bprev ? at(bprev, q.hgl) : T(0);
      hq = qin ? at(qin, q.hgl) : T(0);
    }
    T k18[18];
    gather18(c, nbs, brick, q.lx, q.ly, q.lz, k18, rowm, nb);
    T vs, ws;
    ms_step(v0, w0, j0, ion, dt, vs, ws);
    const T d1 = v0 - b1;
    const T x0 = bprev ? vs + (kd * d1 + q0) : vs;
    s[q.C] = x0;
    if (q.has_halo) {
      T a, b;
      ms_step(hv, hw, hj, ion, dt, a, b);
      s[q.hC] = bprev ? a + (kd * (hv - hb1) + hq) : a;
    }
    ahead.stage(nbt[(m + 1) & 1], rowt[(m + 1) & 1]);
    __syncthreads();
    const T rr = (vs - x0) + dt * apply19(s, q.C, k18);
    // z0 = M^-1 r0, M the diagonal of I - dt A from this voxel's weights
    const T z0 = rr / (T(1) - dt * diag19(k18));
    if (check_prev && vp < theta && theta <= v0) {
      if (isinf(at(tact, q.g))) at(tact, q.g) = static_cast<T>(tprev) + dt * (theta - vp) / (v0 - vp);
    }
    if (!isfinite(v0)) flags[0] = 1;
    if (q.live) {
      st_stream<NT>(&at(x, q.g), x0);
      st_stream<NT>(&at(bout, q.g), vs);
      if (bprev) {
        st_stream<NT>(&at(dout, q.g), d1);
        st_stream<NT>(&at(qout, q.g), q2 * d1 + q3 * d2 + q4 * d3);
      }
      st_stream<NT>(&at(wout, q.g), ws);
      st_stream<NT>(&at(z, q.g), z0);
    }
    const double rd = static_cast<double>(rr);
    acc[0] += static_cast<double>(vs) * static_cast<double>(vs);
    acc[1] += rd * rd;
  }
  block_partials<2>(acc, parts);
}


// k_be_init of FP32 grids, with the pipelined brick loop: the same work and
// results as the template above (the arguments gathered in BeInitArgs); the
// four waves per SIMD asked for keep two blocks resident per CU.
template <bool NT>
__global__ __launch_bounds__(kBV) __attribute__((amdgpu_waves_per_eu(4))) void k_be_init(
    int nb, const int* __restrict__ nbr, CoefSet<float> c, const BeInitArgs A,
    IonicT<float> ion, float dt, float* __restrict__ tact, float theta, double tprev,
    int* flags, CGScalars* cout, double* parts, double tol2, int maxit,
    const uint64_t* __restrict__ rowsn) {
  __shared__ float S0[kIStage], S1[kIStage], s[kTile];
  __shared__ int nbt[2][kNbr];
  __shared__ uint64_t rowt[2][kNbr];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CGScalars st = {};
    st.tol2 = tol2;
    st.maxit = maxit;
    *cout = st;
  }
  be_init_pipelined<NT>(S0, S1, s, nbt, rowt, nb, nbr, rowsn, c, A, ion, dt, tact, theta, tprev,
                        flags, parts);
}

// Status word of a CG launch for the host, written with one 8-byte store to
// coherent pinned host memory (so the host reads it whole without waiting
// for the stream): launch number (high 32 bits), iteration count, fail, done.
__device__ __forceinline__ void publish_status(unsigned long long* mirror, unsigned seq,
                                               const CGScalars& st) {
  if (!mirror) return;
  const unsigned long long v = (static_cast<unsigned long long>(seq) << 32) |
                               (static_cast<unsigned long long>(st.it & 0x3fffffff) << 2) |
                               (static_cast<unsigned long long>(st.fail ? 1 : 0) << 1) |
                               static_cast<unsigned long long>(st.done ? 1 : 0);
  *reinterpret_cast<volatile unsigned long long*>(mirror) = v;
}

// One CG launch.  kind 0: set-up, u0 = M^-1 r0, w0 = K u0 (partials of the
// init launch: (b.b, r.r) when init_kind == 0, or (r.r) with the tolerance
// relative to it when init_kind == 1).  kind 1: first iteration (beta = 0,
// no p / s history).  kind 2: general iteration.  K = c0 I + c1 A.
// Partials: (gamma, delta, rho) = ((r, u), (u, w), (r, r)).
// ---------------------------------------------------------------------------
// Two-level preconditioner of the bidomain inner solve:
//   M^-1 = D^-1 + P Kc^-1 P^T,
// D the diagonal of K, P piecewise constant on aggregates of bricks (a voxel
// of the elliptic domain belongs to its brick's aggregate), Kc = P^T K P with
// s/n_c added to every entry so that it is invertible (K is singular only on
// constants, and the inner solve sees sum-zero residuals, whose restriction
// sums to zero).  Kc^-1 is formed once per conductivity and applied as a
// dense GEMV.  The inner iteration is the one-reduction (Chronopoulos-Gear)
// PCG split over four launches: update (x, r, p, s and the brick sums of r),
// aggregate sums, coarse GEMV, apply (z = M^-1 r, w = K z and the dots).
// Every sum is taken in a fixed order.
// ---------------------------------------------------------------------------

// The 18 off-diagonal entries of the 19-point operator as (offset, sign of
// the weight in gather18's order), apply19's layout.
__device__ __forceinline__ void off18(int i, int& dx, int& dy, int& dz, int& sg) {
  const int o[18][4] = {{1, 0, 0, 1},   {-1, 0, 0, 1},  {0, 1, 0, 1},  {0, -1, 0, 1},
                        {0, 0, 1, 1},   {0, 0, -1, 1},  {1, 1, 0, 1},  {-1, -1, 0, 1},
                        {1, -1, 0, -1}, {-1, 1, 0, -1}, {1, 0, 1, 1},  {-1, 0, -1, 1},
                        {1, 0, -1, -1}, {-1, 0, 1, -1}, {0, 1, 1, 1},  {0, -1, -1, 1},
                        {0, 1, -1, -1}, {0, -1, 1, -1}};
  dx = o[i][0];
  dy = o[i][1];
  dz = o[i][2];
  sg = o[i][3];
}

// Per brick, the 27 sums over the brick's voxels p and the voxels q of
// neighbour slot s of K_pq, K = c0 I + c1 A (FP64 weights), and as a 28th
// value the sum of K's diagonal over the brick.  Block sums in a fixed
// order; kb[brick * kCoarseRow + s].
__global__ __launch_bounds__(kBV) void k_coarse_brick(int nb, const int* __restrict__ nbr,
                                                      CoefSet<double> c, double c0, double c1,
                                                      double* __restrict__ kb) {
  __shared__ int nbs[kNbr];
  __shared__ double red[kBV / 64];
  const int brick = block_brick();
  if (brick >= nb) return;
  const int t = threadIdx.x;
  if (t < kNbr) nbs[t] = nbr[brick * kNbr + t];
  __syncthreads();
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  double k18[18];
  gather18(c, nbs, brick, lx, ly, lz, k18);
  int slot[18];
  double val[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    int dx, dy, dz, sg;
    off18(i, dx, dy, dz, sg);
    const int tx = lx + dx, ty = ly + dy, tz = lz + dz;
    slot[i] = (tx < 0 ? 0 : (tx > 7 ? 2 : 1)) * 9 + (ty < 0 ? 0 : (ty > 7 ? 2 : 1)) * 3 +
              (tz < 0 ? 0 : (tz > 7 ? 2 : 1));
    val[i] = c1 * static_cast<double>(sg) * k18[i];
  }
  const double dg = c0 + c1 * diag19(k18);
  const int lane = t & 63, wave = t >> 6;
  for (int s2 = 0; s2 < kCoarseRow; ++s2) {
    double v = (s2 == 13 || s2 == kNbr) ? dg : 0.0;
    if (s2 < kNbr) {
#pragma unroll
      for (int i = 0; i < 18; ++i) v += (slot[i] == s2) ? val[i] : 0.0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (t == 0) {
      double a = 0.0;
      for (int w = 0; w < kBV / 64; ++w) a += red[w];
      kb[static_cast<int64_t>(brick) * kCoarseRow + s2] = a;
    }
    __syncthreads();
  }
}

// Row I of the dense Kc (n x n, zeroed before): the brick rows of aggregate
// I, its bricks in list order, their 27 slots in order.  One thread per row.
__global__ void k_coarse_rows(int n, const int* __restrict__ agg_ptr,
                              const int* __restrict__ agg_brk, const int* __restrict__ nbr,
                              const int* __restrict__ agg, int nb, const double* __restrict__ kb,
                              double* __restrict__ kc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n) return;
  for (int e = agg_ptr[I]; e < agg_ptr[I + 1]; ++e) {
    const int b = agg_brk[e];
    for (int s2 = 0; s2 < kNbr; ++s2) {
      const int q = nbr[b * kNbr + s2];
      if (q >= nb) continue;
      kc[static_cast<int64_t>(I) * n + agg[q]] += kb[static_cast<int64_t>(b) * kCoarseRow + s2];
    }
  }
}

// a[i] += v for i < len
__global__ void k_add_const(int64_t len, double* __restrict__ a, double v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) a[i] += v;
}

// Blocked Gauss-Jordan inversion in place, no pivoting (Kc is symmetric
// positive definite), kGjPanel columns per step.  With K the step's pivot rows
// and columns, P = A[K,K]:
//   rows K:          A[K,:] <- P^-1 A[K,:],  and A[K,K] <- P^-1;
//   every other row: A[i,:] <- A[i,:] - A[i,K] (P^-1 A[K,:]),  with A[i,K]
//                    taken as 0 on the left, so A[i,K] <- -A[i,K] P^-1.
// Each step reads and writes the matrix once for kGjPanel eliminations.

// P^-1 of the bs x bs pivot block (bs <= kGjPanel) by unblocked Gauss-Jordan in
// LDS, one block of kGjPanel * kGjPanel threads
__global__ __launch_bounds__(kGjPanel * kGjPanel) void k_gj_pivot(int n, const double* __restrict__ a,
                                                          int k0, int bs,
                                                          double* __restrict__ pinv) {
  __shared__ double m[kGjPanel][kGjPanel + 1];
  __shared__ double rowp[kGjPanel], colp[kGjPanel];
  const int r = threadIdx.x / kGjPanel, c = threadIdx.x % kGjPanel;
  const bool in = r < bs && c < bs;
  if (in) m[r][c] = a[static_cast<int64_t>(k0 + r) * n + k0 + c];
  __syncthreads();
  for (int k = 0; k < bs; ++k) {
    if (threadIdx.x < bs) {
      const int t = threadIdx.x;
      const double piv = m[k][k];
      rowp[t] = (t == k ? 1.0 : m[k][t]) / piv;
      colp[t] = (t == k) ? 0.0 : m[t][k];
    }
    __syncthreads();
    if (in) m[r][c] = (r == k) ? rowp[c] : (c == k ? 0.0 : m[r][c]) - colp[r] * rowp[c];
    __syncthreads();
  }
  if (in) pinv[r * kGjPanel + c] = m[r][c];
}

// Row panel rp[t][j] = (P^-1 A[K,:])[t][j] for j outside K, P^-1[t][j - k0]
// inside; column panel cp[i][t] = A[i][k0 + t] (i outside K; 0 inside)
__global__ void k_gj_panels(int n, const double* __restrict__ a, int k0, int bs,
                            const double* __restrict__ pinv, double* __restrict__ rp,
                            double* __restrict__ cp) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(kGjPanel) * n) return;
  const int t = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  if (t < bs) {
    double v;
    if (j >= k0 && j < k0 + bs) {
      v = pinv[t * kGjPanel + (j - k0)];
    } else {
      v = 0.0;
      for (int u = 0; u < bs; ++u) v += pinv[t * kGjPanel + u] * a[static_cast<int64_t>(k0 + u) * n + j];
    }
    rp[static_cast<int64_t>(t) * n + j] = v;
    // the same thread grid also copies column t of the pivot columns (row j)
    cp[static_cast<int64_t>(j) * kGjPanel + t] =
        (j >= k0 && j < k0 + bs) ? 0.0 : a[static_cast<int64_t>(j) * n + k0 + t];
  }
}

// The rank-bs update of one 16 x 16 tile of A per block: panel slices in LDS
__global__ __launch_bounds__(256) void k_gj_update(int n, double* __restrict__ a, int k0, int bs,
                                                   const double* __restrict__ rp,
                                                   const double* __restrict__ cp) {
  __shared__ double cs[16][kGjPanel + 1], rs[kGjPanel][17];
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  for (int e = threadIdx.x; e < 16 * kGjPanel; e += 256) {
    const int r = e / kGjPanel, t = e % kGjPanel;
    cs[r][t] = (i0 + r < n && t < bs) ? cp[static_cast<int64_t>(i0 + r) * kGjPanel + t] : 0.0;
    const int t2 = e / 16, c2 = e % 16;
    rs[t2][c2] = (j0 + c2 < n && t2 < bs) ? rp[static_cast<int64_t>(t2) * n + j0 + c2] : 0.0;
  }
  __syncthreads();
  const int i = i0 + ti, j = j0 + tj;
  if (i >= n || j >= n) return;
  const int64_t idx = static_cast<int64_t>(i) * n + j;
  if (i >= k0 && i < k0 + bs) {
    a[idx] = rs[i - k0][tj];
    return;
  }
  double acc = 0.0;
  for (int t = 0; t < bs; ++t) acc += cs[ti][t] * rs[t][tj];
  a[idx] = ((j >= k0 && j < k0 + bs) ? 0.0 : a[idx]) - acc;
}

// FP32 copy of the n x n inverse with rows padded to ld (a multiple of 4)
// FP16 copy of the coarse inverse for the GEMV, scaled by `scale` (chosen so
// that the largest entry, on the diagonal of this SPD matrix, maps to 2^14),
// rows padded to ld with zeros
__global__ void k_to_f16(int n, int ld, const double* __restrict__ a, double scale,
                         _Float16* __restrict__ o) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * ld) return;
  const int i = static_cast<int>(idx / ld), j = static_cast<int>(idx % ld);
  o[idx] = j < n ? static_cast<_Float16>(static_cast<float>(a[static_cast<int64_t>(i) * n + j] *
                                                            scale))
                 : static_cast<_Float16>(0.0f);
}

// Update launch of the two-level inner PCG.  kind 0 (first): the scalars
// from the inner init's (r, r) partials, no vector update.  kind 1: the
// convergence test on (r, r) of the last apply, then alpha, beta from its
// (r, z) and (z, w) and
//   p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s.
// Both write the brick sums of r for the restriction.
__global__ __launch_bounds__(kBV) void k_cg2_update(
    int nb, float* __restrict__ x, float* __restrict__ r, float* __restrict__ p,
    float* __restrict__ s, const float* __restrict__ z, const float* __restrict__ w,
    float* __restrict__ rb, int kind, const CGScalars* __restrict__ cin, CGScalars* cout,
    const double* __restrict__ prev, unsigned long long* mirror, unsigned seq) {
  const CGScalars in = *cin;
  if (in.done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *cout = in;
      publish_status(mirror, seq, in);
    }
    return;
  }
  CGScalars st = in;
  bool upd = false;
  if (kind == 0) {
    double S[1];
    sum_prev<1>(prev, gridDim.x, S);
    st.bb = S[0];
    st.rr = S[0];
    st.it = 0;
    st.fail = 0;
    st.alpha = st.beta = st.rz = 0.0;
    st.done = (S[0] == 0.0) ? 1 : 0;
  } else {
    double S[3];
    sum_prev<3>(prev, gridDim.x, S);
    const double gam = S[0], del = S[1], rho = S[2];
    st.rr = rho;
    if (!isfinite(rho)) { st.done = 1; st.fail = 1; }
    else if (rho <= in.tol2 * in.bb) st.done = 1;
    else if (in.it >= in.maxit) { st.done = 1; st.fail = 1; }
    else if (!(gam > 0.0)) { st.done = 1; st.fail = 1; }   // M not positive definite
    else {
      const double beta = (in.it == 0) ? 0.0 : gam / in.rz;
      const double den = (in.it == 0) ? del : del - beta * gam / in.alpha;
      if (!(den > 0.0) || !isfinite(den)) { st.done = 1; st.fail = 1; }
      else {
        st.beta = beta;
        st.alpha = gam / den;
        st.rz = gam;
        st.it = in.it + 1;
        upd = true;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *cout = st;
    publish_status(mirror, seq, st);
  }
  if (st.done) return;
  __shared__ float red[kBV / 64];
  const float alpha = static_cast<float>(st.alpha), beta = static_cast<float>(st.beta);
  const bool first = in.it == 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 0;; ++m) {
    const int brick = pbrick(m, nb);
    if (brick < 0) break;
    const int g = brick * kBV + threadIdx.x;
    float rn = r[g];
    if (upd) {
      const float pn = first ? z[g] : z[g] + beta * p[g];
      const float sn = first ? w[g] : w[g] + beta * s[g];
      p[g] = pn;
      s[g] = sn;
      x[g] += alpha * pn;
      rn -= alpha * sn;
      r[g] = rn;
    }
    float v = rn;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      float a = 0.0f;
      for (int k = 0; k < kBV / 64; ++k) a += red[k];
      rb[brick] = a;
    }
    __syncthreads();
  }
}

// rc[I] = sum of the brick sums of aggregate I, in list order
__global__ void k_agg_sum(int n, const int* __restrict__ agg_ptr, const int* __restrict__ agg_brk,
                          const float* __restrict__ rb, float* __restrict__ rc,
                          const CGScalars* __restrict__ st) {
  if (st->done) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n) return;
  float a = 0.0f;
  for (int e = agg_ptr[I]; e < agg_ptr[I + 1]; ++e) a += rb[agg_brk[e]];
  rc[I] = a;
}

// cc[I] = unscale * sum_J kinv[I][J] rc[J] from the scaled FP16 inverse:
// one block per row, rows padded to ld (rc zero beyond n), 8-byte loads of
// four entries, FP64 accumulation
__global__ __launch_bounds__(256) void k_coarse_gemv(int ld, const _Float16* __restrict__ kinv,
                                                     float unscale,
                                                     const float* __restrict__ rc,
                                                     float* __restrict__ cc,
                                                     const CGScalars* __restrict__ st) {
  if (st->done) return;
  __shared__ double red[4];
  typedef float F4 __attribute__((ext_vector_type(4)));
  typedef _Float16 H4 __attribute__((ext_vector_type(4)));
  const int I = blockIdx.x;
  const H4* row = reinterpret_cast<const H4*>(kinv + static_cast<int64_t>(I) * ld);
  const F4* v = reinterpret_cast<const F4*>(rc);
  double a = 0.0;
  for (int j = threadIdx.x; j < ld / 4; j += 256) {
    const H4 h = row[j];
    const F4 x = v[j];
    const float m0 = static_cast<float>(h.x), m1 = static_cast<float>(h.y);
    const float m2 = static_cast<float>(h.z), m3 = static_cast<float>(h.w);
    a += static_cast<double>(m0 * x.x + m1 * x.y) + static_cast<double>(m2 * x.z + m3 * x.w);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0)
    cc[I] = static_cast<float>((red[0] + red[1] + red[2] + red[3]) * static_cast<double>(unscale));
}

// Apply launch: z = D^-1 r + P cc on the elliptic domain (where D^-1 > 0),
// w = c0 z + c1 A z, and the partials (r, z), (z, w), (r, r).  Every voxel
// of the brick is written.
__global__ __launch_bounds__(kBV) void k_cg2_apply(
    int nb, const int* __restrict__ nbr, CoefSet<float> c, float c0, float c1,
    const float* __restrict__ dinv, const float* __restrict__ r, const float* __restrict__ cc,
    const int* __restrict__ agg, float* __restrict__ z, float* __restrict__ w,
    const CGScalars* __restrict__ cin, double* parts, const uint64_t* __restrict__ rowsn) {
  if (cin->done) return;
  __shared__ float s[kTile];
  __shared__ int nbt[2][kNbr];
  __shared__ uint64_t rowt[2][kNbr];
  double acc[3] = {0.0, 0.0, 0.0};
  NbrAhead ahead;
  int nxt = pbrick(0, nb);
  ahead.fetch(nbr, rowsn, nxt);
  ahead.stage(nbt[0], rowt[0]);
  for (int m = 0; nxt >= 0; ++m) {
    const int brick = nxt;
    const int* nbs = nbt[m & 1];
    nxt = pbrick(m + 1, nb);
    ahead.fetch(nbr, rowsn, nxt);
    __syncthreads();
    const Cell e = cell_setup(nbs, brick);
    const float rg = at(r, e.g), dg = at(dinv, e.g);
    const float cown = cc[agg[brick]];
    float hr = 0.0f, hd = 0.0f, hc = 0.0f;
    if (e.has_halo) {
      hr = at(r, e.hg);
      hd = at(dinv, e.hg);
      hc = cc[agg[e.hg / kBV]];
    }
    float k18[18];
    gather18(c, nbs, brick, e.lx, e.ly, e.lz, k18);
    const float zn = dg > 0.0f ? dg * rg + cown : 0.0f;
    s[e.C] = zn;
    if (e.has_halo) s[e.hC] = hd > 0.0f ? hd * hr + hc : 0.0f;
    ahead.stage(nbt[(m + 1) & 1], rowt[(m + 1) & 1]);
    __syncthreads();
    const float wv = c0 * zn + c1 * apply19(s, e.C, k18);
    at(z, e.g) = zn;
    at(w, e.g) = wv;
    acc[0] += static_cast<double>(rg) * static_cast<double>(zn);
    acc[1] += static_cast<double>(zn) * static_cast<double>(wv);
    acc[2] += static_cast<double>(rg) * static_cast<double>(rg);
  }
  block_partials<3>(acc, parts);
}

// Four consecutive voxels of a brick row (16 B in FP32), loaded and stored
// as one vector access.
template <typename T> struct Quad {
  typedef T V __attribute__((ext_vector_type(4)));
};

// Jacobi-PCG with one launch per iteration and no set-up apply: the
// textbook recurrences, with the next residual's two norms, (r, z) and
// (r, r), expanded in dot products of the previous launch's own vectors, so
// that the x / r update, the new direction and the operator apply of one
// iteration share a launch.  K = c0 I + c1 A, M its diagonal (from each
// voxel's own weights), z = M^-1 r.  The solve keeps z and t = M^-1 q
// instead of r and q: z' = z - alpha t and q' = K p' = K z' + beta q follow
// from the recurrences, so the operator is applied to z' and the only
// vectors read at the halo are z and t (r = M z and q = M t are formed
// pointwise where needed, and no diagonal array is read).
//   launch 0: tests the init's residual ((b.b, r.r) partials), then
//     p_0 = z_0, q_0 = K z_0, t_0 = M^-1 q_0 (z_0 stays where the init left it);
//   launch k >= 1: from launch k-1's dots, alpha = gamma / delta,
//     gamma' = gamma - 2 alpha (q, z) + alpha^2 (q, M^-1 q),
//     rho'   = rho   - 2 alpha (q, r) + alpha^2 (q, q).
//     If rho' <= tol^2 (b, b) the solve is done and only x += alpha p is
//     left: a pointwise pass (also taken when maxit is reached, flagged as
//     failed).  Otherwise x += alpha p, z' = z - alpha t, beta = gamma' /
//     gamma, p' = z' + beta p, q' = K z' + beta M t, t' = M^-1 q'.
// The dots are accumulated in FP64 from the FP32 vectors, so the expansion
// loses nothing that matters next to the FP32 rounding of r' itself.
// Partials: (delta, gamma, (q, z), (q, M^-1 q), rho, (q, r), (q, q)) of the
// launch's own p, q, r, z, t.  z and t are read at the halo and p by the
// next launch, so a launch writes the other buffer of each pair; x is
// updated in place.
template <typename T, bool NT>
__global__ __launch_bounds__(kBV) __attribute__((amdgpu_waves_per_eu(4))) void k_pcg_step(
    int nb, const int* __restrict__ nbr, CoefSet<T> c, T c0, T c1, T* __restrict__ x,
    const T* __restrict__ z_in, T* __restrict__ z_out, const T* __restrict__ p_in,
    T* __restrict__ p_out, const T* __restrict__ t_in, T* __restrict__ t_out, int first,
    const CGScalars* __restrict__ cin, CGScalars* cout, const double* __restrict__ prev,
    double* parts, const uint64_t* __restrict__ rowsn, unsigned long long* mirror,
    unsigned seq) {
  const CGScalars in = *cin;
  if (in.done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *cout = in;
      publish_status(mirror, seq, in);
    }
    return;
  }
  CGScalars st = in;
  bool final_x = false;
  if (first) {
    double S[2];
    sum_prev<2>(prev, gridDim.x, S);
    st.bb = S[0];
    st.rr = S[1];
    st.it = 0;
    st.fail = 0;
    st.alpha = 0.0;
    st.beta = 0.0;
    st.done = (S[0] == 0.0 || S[1] <= in.tol2 * S[0]) ? 1 : 0;
  } else {
    double S[7];
    sum_prev<7>(prev, gridDim.x, S);
    const double del = S[0], gam = S[1], qz = S[2], qmq = S[3], rho = S[4], qr = S[5],
                 qq = S[6];
    st.it = in.it + 1;
    if (!(del > 0.0) || !isfinite(del) || !isfinite(gam)) {
      st.done = 1;
      st.fail = 1;
    } else {
      const double alpha = gam / del;
      const double gam1 = gam - 2.0 * alpha * qz + alpha * alpha * qmq;
      const double rho1 = rho - 2.0 * alpha * qr + alpha * alpha * qq;
      st.alpha = alpha;
      st.rr = rho1;
      if (!isfinite(rho1) || !isfinite(gam1)) {
        st.done = 1;
        st.fail = 1;
      } else if (rho1 <= in.tol2 * in.bb) {
        st.done = 1;
        final_x = true;
      } else if (st.it >= in.maxit || !(gam1 > 0.0)) {
        st.done = 1;
        st.fail = 1;
        final_x = true;
      } else {
        st.beta = gam1 / gam;
        st.rz = gam1;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *cout = st;
    publish_status(mirror, seq, st);
  }
  const T alpha = static_cast<T>(st.alpha), beta = static_cast<T>(st.beta);
  if (final_x) {
    // the last x update, pointwise over the rows holding tissue: half a row
    // (4 voxels, vector accesses) per thread, 4 bricks per block at a time
    using V = typename Quad<T>::V;
    const int slot = threadIdx.x >> 7;
    const int e = (threadIdx.x & 127) * 4;
    const int bit = e >> 3;
    for (int m = slot;; m += 4) {
      const int brick = pbrick(m, nb);
      if (brick < 0) break;
      if ((rowsn[brick * kNbr + 13] >> bit) & 1) {
        const int g = brick * kBV + e;
        const V xv = ld_stream<NT>(reinterpret_cast<const V*>(x + g));
        const V pv = ld_stream<NT>(reinterpret_cast<const V*>(p_in + g));
        st_stream<NT>(reinterpret_cast<V*>(x + g), xv + alpha * pv);
      }
    }
    return;
  }
  if (st.done) return;
  if constexpr (sizeof(T) == 4) {
    __shared__ float S0[kStage], S1[kStage], s[kTile];
    __shared__ int nbt[2][kNbr];
    __shared__ uint64_t rowt[2][kNbr];
    if (first)
      pcg_iter_pipelined<NT, true>(S0, S1, s, nbt, rowt, nb, nbr, rowsn, c, c0, c1, alpha, beta,
                                   x, z_in, z_out, p_in, p_out, t_in, t_out, parts);
    else
      pcg_iter_pipelined<NT, false>(S0, S1, s, nbt, rowt, nb, nbr, rowsn, c, c0, c1, alpha,
                                    beta, x, z_in, z_out, p_in, p_out, t_in, t_out, parts);
    return;
  } else {
  __shared__ T s[kTile];
  __shared__ int nbt[2][kNbr];
  __shared__ uint64_t rowt[2][kNbr];
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  NbrAhead ahead;
  int nxt = pbrick(0, nb);
  ahead.fetch(nbr, rowsn, nxt);
  ahead.stage(nbt[0], rowt[0]);
  for (int m = 0; nxt >= 0; ++m) {
    const int brick = nxt;
    const int* nbs = nbt[m & 1];
    const uint64_t* rowm = rowt[m & 1];
    nxt = pbrick(m + 1, nb);
    ahead.fetch(nbr, rowsn, nxt);
    __syncthreads();
    const Cell e = cell_setup(nbs, brick, rowm, nb);
    const T zg = at(z_in, e.gl);
    const T tg = first ? T(0) : at(t_in, e.gl);
    const T pg = first ? T(0) : at(p_in, e.gl);
    const T xg = first ? T(0) : ld_stream<NT>(&at(x, e.gl));
    T hz = T(0), ht = T(0);
    if (e.has_halo) {
      hz = at(z_in, e.hgl);
      ht = first ? T(0) : at(t_in, e.hgl);
    }
    T k18[18];
    gather18(c, nbs, brick, e.lx, e.ly, e.lz, k18, rowm, nb);
    // z_k = z_{k-1} - alpha t_{k-1} on the brick and its halo
    const T zn = zg - alpha * tg;
    s[e.C] = zn;
    if (e.has_halo) s[e.hC] = hz - alpha * ht;
    ahead.stage(nbt[(m + 1) & 1], rowt[(m + 1) & 1]);
    __syncthreads();
    // q_k = K p_k = K z_k + beta q_{k-1}, with q_{k-1} = M t_{k-1}
    const T md = c0 + c1 * diag19(k18);
    const T qn = (c0 * zn + c1 * apply19(s, e.C, k18)) + beta * (md * tg);
    const T pn = zn + beta * pg;
    const T tn = qn / md;
    const T rn = md * zn;
    if (e.live) {
      if (!first) {
        st_stream<NT>(&at(x, e.g), xg + alpha * pg);
        st_stream<NT>(&at(z_out, e.g), zn);
      }
      st_stream<NT>(&at(p_out, e.g), pn);
      st_stream<NT>(&at(t_out, e.g), tn);
    }
    const double dr = rn, dz = zn, dp = pn, dq = qn;
    acc[0] += dp * dq;
    acc[1] += dr * dz;
    acc[2] += dq * dz;
    acc[3] += dq * static_cast<double>(tn);
    acc[4] += dr * dr;
    acc[5] += dq * dr;
    acc[6] += dq * dq;
  }
  block_partials<7>(acc, parts);
  }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ partials,
                                                       int nparts, int K, double* out) {
  __shared__ double sm[3][kRedThreads];
  const int t = threadIdx.x;
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = t; i < nparts; i += kRedThreads) s += partials[k * nparts + i];
    sm[k][t] = s;
  }
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < K; ++k) sm[k][t] += sm[k][t + w];
    __syncthreads();
  }
  if (t == 0)
    for (int k = 0; k < K; ++k) out[k] = sm[k][0];
}

template <typename T>
__global__ __launch_bounds__(kBV) void k_activation(int nb, const T* __restrict__ vold,
                                                    const T* __restrict__ vnew,
                                                    T* __restrict__ tact, T dt, T theta,
                                                    double tn, int* flags) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  const T v0 = vold[g], vn = vnew[g];
  if (v0 < theta && theta <= vn) {
    if (isinf(tact[g])) tact[g] = static_cast<T>(tn) + dt * (theta - v0) / (vn - v0);
  }
  if (!isfinite(vn)) flags[0] = 1;
}

// One Jacobi sweep of the implicit-Euler system (I - dt A) x = b, the
// thesis's own solver (Linear Solver section, "Implicit Euler",
// eqn:iejac1): x_out = x + M^-1 (b - (I - dt A) x) with M = diag(I - dt A),
// which is [I - dt D]^-1 [b + dt (L + U) x] rewritten.  One brick per block,
// no reductions; rows without tissue read the ghost brick and are not
// stored.
template <typename T>
__global__ __launch_bounds__(kBV) void k_jacobi(int nb, const int* __restrict__ nbr,
                                                CoefSet<T> c, T dt, const T* __restrict__ dinv,
                                                const T* __restrict__ b,
                                                const T* __restrict__ x_in,
                                                T* __restrict__ x_out,
                                                const uint64_t* __restrict__ rowsn) {
  __shared__ T s[kTile];
  __shared__ int nbs[kNbr];
  __shared__ uint64_t rowm[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  if (threadIdx.x < kNbr) {
    nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
    rowm[threadIdx.x] = rowsn[brick * kNbr + threadIdx.x];
  }
  __syncthreads();
  const Cell e = cell_setup(nbs, brick, rowm, nb);
  const T xg = at(x_in, e.gl), bg = at(b, e.gl), dg = at(dinv, e.gl);
  s[e.C] = xg;
  if (e.has_halo) s[e.hC] = at(x_in, e.hgl);
  T k18[18];
  gather18(c, nbs, brick, e.lx, e.ly, e.lz, k18, rowm, nb);
  __syncthreads();
  const T r = (bg - xg) + dt * apply19(s, e.C, k18);
  if (e.live) at(x_out, e.g) = xg + dg * r;
}

// Jacobi: dinv = 1 / (c0 + c1 A_pp) where positive, else 0.
template <typename T>
__global__ __launch_bounds__(kBV) void k_dinv(int nb, const int* __restrict__ nbr, CoefSet<T> c,
                                              T c0, T c1, T* __restrict__ dinv) {
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  const int t = threadIdx.x;
  if (t < kNbr) nbs[t] = nbr[brick * kNbr + t];
  __syncthreads();
  const int lx = t >> 6, ly = (t >> 3) & 7, lz = t & 7;
  T k18[18];
  gather18(c, nbs, brick, lx, ly, lz, k18);
  const T d = c0 + c1 * diag19(k18);
  dinv[brick * kBV + t] = d > T(0) ? T(1) / d : T(0);
}

template <typename T>
__global__ __launch_bounds__(kBV) void k_sum(int nb, const T* __restrict__ x, double* partials) {
  const int brick = block_brick();
  if (brick >= nb) { idle_partials<1>(partials); return; }
  double acc[1] = {static_cast<double>(x[brick * kBV + threadIdx.x])};
  block_partials<1>(acc, partials);
}

// scatter the current stimulus currents; qstep = sum of the values (FP64)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_stim_scatter(const int64_t* __restrict__ idx,
                                                             const double* __restrict__ val,
                                                             int n, T* __restrict__ jstim,
                                                             double* qstep) {
  __shared__ double sm[kRedThreads];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int i = t; i < n; i += kRedThreads) {
    jstim[idx[i]] = static_cast<T>(val[i]);
    s += val[i];
  }
  sm[t] = s;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (t < w) sm[t] += sm[t + w];
    __syncthreads();
  }
  if (t == 0) qstep[0] = sm[0];
}

__global__ void k_q_accum(double* qacc, const double* qstep, double scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) qacc[0] += scale * qstep[0];
}

// ---------------------------------------------------------------------------
// bidomain
// ---------------------------------------------------------------------------
// r = b - K phi in FP64 with b = A_i v* and K = -(A_i + A_e) (coefficient set
// ck holds A_i + A_e).  Partials: (r.r, sum r, b.b).
template <typename T>
__global__ __launch_bounds__(kBV) void k_resid64(int nb, const int* __restrict__ nbr,
                                                 CoefSet<double> ci, CoefSet<double> ck,
                                                 const T* __restrict__ vs,
                                                 const double* __restrict__ phi,
                                                 double* __restrict__ r64, double* partials) {
  __shared__ double sa[kTile];
  __shared__ double sb[kTile];
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) { idle_partials<3>(partials); return; }
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  sa[q.C] = static_cast<double>(at(vs, q.g));
  sb[q.C] = at(phi, q.g);
  if (q.has_halo) {
    sa[q.hC] = static_cast<double>(at(vs, q.hg));
    sb[q.hC] = at(phi, q.hg);
  }
  __syncthreads();
  double k18[18];
  gather18(ci, nbs, brick, q.lx, q.ly, q.lz, k18);
  const double b = apply19(sa, q.C, k18);
  gather18(ck, nbs, brick, q.lx, q.ly, q.lz, k18);
  const double r = b + apply19(sb, q.C, k18);
  at(r64, q.g) = r;
  double acc[3] = {r * r, r, b * b};
  block_partials<3>(acc, partials);
}

// inner solve start: r32 = (r64 - mean) on tissue, x32 = 0.  Persistent
// like the CG kernels; partial (r.r).
__global__ __launch_bounds__(kBV) void k_inner_init(int nb, const double* __restrict__ r64,
                                                    const uint8_t* __restrict__ mask,
                                                    const double* __restrict__ sums,
                                                    double inv_count, float* __restrict__ x,
                                                    float* __restrict__ r, CGScalars* cout,
                                                    double* parts, double tol2, int maxit) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CGScalars st = {};
    st.tol2 = tol2;
    st.maxit = maxit;
    *cout = st;
  }
  const double mean = sums[1] * inv_count;
  double acc[1] = {0.0};
  for (int m = 0;; ++m) {
    const int brick = pbrick(m, nb);
    if (brick < 0) break;
    const int g = brick * kBV + threadIdx.x;
    const float rv = mask[g] ? static_cast<float>(r64[g] - mean) : 0.0f;
    r[g] = rv;
    x[g] = 0.0f;
    const double rd = static_cast<double>(rv);
    acc[0] += rd * rd;
  }
  block_partials<1>(acc, parts);
}

// phi += d (FP64); partial sum of phi
__global__ __launch_bounds__(kBV) void k_phi_correct(int nb, double* __restrict__ phi,
                                                     const float* __restrict__ d,
                                                     const uint8_t* __restrict__ mask,
                                                     double* partials) {
  const int brick = block_brick();
  if (brick >= nb) { idle_partials<1>(partials); return; }
  const int g = brick * kBV + threadIdx.x;
  const double p = mask[g] ? phi[g] + static_cast<double>(d[g]) : 0.0;
  phi[g] = p;
  double acc[1] = {p};
  block_partials<1>(acc, partials);
}

__global__ __launch_bounds__(kBV) void k_phi_shift(int nb, double* __restrict__ phi,
                                                   const uint8_t* __restrict__ mask,
                                                   const double* __restrict__ sum,
                                                   double inv_count) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  const double mean = sum[0] * inv_count;
  phi[g] = mask[g] ? phi[g] - mean : 0.0;
}

// Initial guess of the next elliptic solve: the polynomial in time through
// the last solutions h1 (newest), h2, h3: phi = 2 h1 - h2 (order 2) or
// 3 h1 - 3 h2 + h3 (order 3).  The weights sum to 1, so sum phi = 0 holds.
__global__ __launch_bounds__(kBV) void k_phi_extrap(int nb, double* __restrict__ phi,
                                                    const double* __restrict__ h1,
                                                    const double* __restrict__ h2,
                                                    const double* __restrict__ h3, int order) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  phi[g] = order >= 3 ? 3.0 * (h1[g] - h2[g]) + h3[g] : 2.0 * h1[g] - h2[g];
}

// v_{n+1} = v* + dt A_i (v* + phi), with the activation check
template <typename T>
__global__ __launch_bounds__(kBV) void k_parabolic(int nb, const int* __restrict__ nbr,
                                                   CoefSet<T> ci, const T* __restrict__ vs,
                                                   const double* __restrict__ phi,
                                                   const T* __restrict__ vold,
                                                   T* __restrict__ vout, T* __restrict__ tact,
                                                   T dt, T theta, double tn, int* flags) {
  __shared__ T s[kTile];
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  const T vsg = at(vs, q.g);
  const double pg = at(phi, q.g);
  const T v0 = at(vold, q.g);
  T hv = T(0);
  double hp = 0.0;
  if (q.has_halo) {
    hv = at(vs, q.hg);
    hp = at(phi, q.hg);
  }
  T k18[18];
  gather18(ci, nbs, brick, q.lx, q.ly, q.lz, k18);
  s[q.C] = vsg + static_cast<T>(pg);
  if (q.has_halo) s[q.hC] = hv + static_cast<T>(hp);
  __syncthreads();
  const T vn = vsg + dt * apply19(s, q.C, k18);
  at(vout, q.g) = vn;
  if (v0 < theta && theta <= vn) {
    if (isinf(at(tact, q.g))) at(tact, q.g) = static_cast<T>(tn) + dt * (theta - v0) / (vn - v0);
  }
  if (!isfinite(vn)) flags[0] = 1;
}

// y = A x; partials (y.y, x.y)
template <typename T>
__global__ __launch_bounds__(kBV) void k_apply(int nb, const int* __restrict__ nbr, CoefSet<T> c,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               double* partials) {
  __shared__ T s[kTile];
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) { idle_partials<2>(partials); return; }
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  const T xg = at(x, q.g);
  s[q.C] = xg;
  if (q.has_halo) s[q.hC] = at(x, q.hg);
  T k18[18];
  gather18(c, nbs, brick, q.lx, q.ly, q.lz, k18);
  __syncthreads();
  const T yv = apply19(s, q.C, k18);
  at(y, q.g) = yv;
  double acc[2] = {static_cast<double>(yv) * static_cast<double>(yv),
                   static_cast<double>(xg) * static_cast<double>(yv)};
  if (partials) block_partials<2>(acc, partials);
}

// Per-block maximum of the Gershgorin row bound |A_pp| + sum_q |A_pq|.
__global__ __launch_bounds__(kBV) void k_block_max(int nb, const int* __restrict__ nbr,
                                                   CoefSet<double> c, double* partials) {
  __shared__ int nbs[kNbr];
  __shared__ double red[kBV / 64];
  const int brick = block_brick();
  if (brick >= nb) { if (threadIdx.x == 0) partials[blockIdx.x] = 0.0; return; }
  const int t = threadIdx.x;
  if (t < kNbr) nbs[t] = nbr[brick * kNbr + t];
  __syncthreads();
  double k18[18];
  gather18(c, nbs, brick, t >> 6, (t >> 3) & 7, t & 7, k18);
  double gsum = fabs(diag19(k18));
  for (int i = 0; i < 18; ++i) gsum += fabs(k18[i]);
  for (int off = 32; off > 0; off >>= 1) gsum = fmax(gsum, __shfl_xor(gsum, off, 64));
  if ((t & 63) == 0) red[t >> 6] = gsum;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int i = 0; i < kBV / 64; ++i) m = fmax(m, red[i]);
    partials[blockIdx.x] = m;
  }
}

// x = y / sqrt(sums[0]) (power iteration normalisation)
__global__ __launch_bounds__(kBV) void k_scale(int nb, double* __restrict__ x,
                                               const double* __restrict__ y,
                                               const double* __restrict__ sums) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  const double n2 = sums[0];
  x[g] = n2 > 0.0 ? y[g] / sqrt(n2) : 0.0;
}

// ---------------------------------------------------------------------------
// discrete adjoint of the explicit monodomain step (reverse mode)
// ---------------------------------------------------------------------------
// Forward step n: v* = v + dt f(v, w) (+ J_stim), w' = w + dt g(v, w),
// v_{n+1} = (I + dt A(s)) v*, with A symmetric and the voxel tensors
// s_q D0_q.  Activation times T enter the loss sum (T - T*)^2.
//
// Adjoint step n maps (lv, lw) = dL/d(v_{n+1}, w_{n+1}) to dL/d(v_n, w_n):
//   nu   = lv + dt A lv                                   ((I + dt A)^T)
//   grad_q += -dt dB(lv, v*)/ds_q   (B: bilinear form of the energy; faces
//             touching q carry D0_q / 2, 2x2 blocks D0_q / 4)
//   lv_n = nu dv*/dv + (direct dT/dv_n of crossings at steps n and n-1)
//   lw_n = nu dv*/dw + lw dw'/dw  (the gate switch is a Dirac, dropped)

// dB(mu, u)/ds_q at tile cell C for voxel tensor d0 (xx, yy, zz, xy, xz, yz)
template <typename T>
__device__ __forceinline__ T dB_ds(const T* sm, const T* su, const uint8_t* mk, int C,
                                   const T d0[6], T inv_h2) {
  T acc = T(0);
  const int off[3] = {100, 10, 1};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
      const int Q = C + sg * off[d];
      if (mk[C] && mk[Q])
        acc += T(0.5) * d0[d] * (sm[Q] - sm[C]) * (su[Q] - su[C]) * inv_h2;
    }
  }
  const int pd[3] = {0, 0, 1}, pe[3] = {1, 2, 2};
#pragma unroll
  for (int pl = 0; pl < 3; ++pl) {
    const int od = off[pd[pl]], oe = off[pe[pl]];
#pragma unroll
    for (int ad = 0; ad <= 1; ++ad) {
#pragma unroll
      for (int ae = 0; ae <= 1; ++ae) {
        const int b0 = C - ad * od - ae * oe;
        const int b1 = b0 + od, b2 = b0 + oe, b3 = b0 + od + oe;
        if (!(mk[b0] && mk[b1] && mk[b2] && mk[b3])) continue;
        const T gdm = sm[b1] + sm[b3] - sm[b0] - sm[b2];
        const T gem = sm[b2] + sm[b3] - sm[b0] - sm[b1];
        const T gdu = su[b1] + su[b3] - su[b0] - su[b2];
        const T geu = su[b2] + su[b3] - su[b0] - su[b1];
        acc += T(0.25) * d0[3 + pl] * (gdm * geu + gdu * gem) * (T(0.25) * inv_h2);
      }
    }
  }
  return acc;
}

// dT/dv seed of a voxel that crossed theta at step `cs`: T depends on
// v_cs (before) and v_cs+1 (after).
template <typename T>
__device__ __forceinline__ T cross_seed(T vb, T va, T theta, T dt, T dl, bool before) {
  const T del = va - vb;
  return before ? dl * (dt * (theta - va) / (del * del))
                : dl * (-dt * (theta - vb) / (del * del));
}

// lv_N = seeds of crossings at step N-1 (dT/dv_N), lw_N = 0
template <typename T>
__global__ __launch_bounds__(kBV) void k_adj_init(int nb, const uint8_t* __restrict__ mask,
                                                  const T* __restrict__ vlast,
                                                  const T* __restrict__ vprev,
                                                  const int* __restrict__ cross,
                                                  const T* __restrict__ tact,
                                                  const T* __restrict__ tstar, T* __restrict__ lv,
                                                  T* __restrict__ lw, T dt, T theta, int nlast) {
  const int brick = block_brick();
  if (brick >= nb) return;
  const int g = brick * kBV + threadIdx.x;
  T a = T(0);
  if (mask[g] && cross[g] == nlast && isfinite(tstar[g]))
    a = cross_seed(vprev[g], vlast[g], theta, dt, T(2) * (tact[g] - tstar[g]), false);
  lv[g] = a;
  lw[g] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kBV) void k_adj_step(
    int nb, const int* __restrict__ nbr, CoefSet<T> c, CoefSet<T> d0,
    const uint8_t* __restrict__ mask, const T* __restrict__ lv_in, const T* __restrict__ lw_in,
    T* __restrict__ lv_out, T* __restrict__ lw_out, const T* __restrict__ v,
    const T* __restrict__ w, const T* __restrict__ jstim, const T* __restrict__ vnext,
    const T* __restrict__ vprev, const int* __restrict__ cross, const T* __restrict__ tact,
    const T* __restrict__ tstar, double* __restrict__ grad, IonicT<T> ion, T dt, T theta,
    T inv_h2, int n) {
  __shared__ T sm[kTile];
  __shared__ T su[kTile];
  __shared__ uint8_t mk[kTile];
  __shared__ int nbs[kNbr];
  const int brick = block_brick();
  if (brick >= nb) return;
  if (threadIdx.x < kNbr) nbs[threadIdx.x] = nbr[brick * kNbr + threadIdx.x];
  __syncthreads();
  const Cell q = cell_setup(nbs, brick);
  const T mu = at(lv_in, q.g), v0 = at(v, q.g), w0 = at(w, q.g);
  const T j0 = jstim ? at(jstim, q.g) : T(0);
  const uint8_t m0 = at(mask, q.g);
  T hm = T(0), hv = T(0), hw = T(0), hj = T(0);
  uint8_t hk = 0;
  if (q.has_halo) {
    hm = at(lv_in, q.hg);
    hv = at(v, q.hg);
    hw = at(w, q.hg);
    hj = jstim ? at(jstim, q.hg) : T(0);
    hk = at(mask, q.hg);
  }
  T k18[18];
  gather18(c, nbs, brick, q.lx, q.ly, q.lz, k18);
  T dq[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) dq[k] = d0.c[k][q.g];
  T vs, ws;
  ms_step(v0, w0, j0, ion, dt, vs, ws);
  sm[q.C] = mu;
  su[q.C] = vs;
  mk[q.C] = m0;
  if (q.has_halo) {
    T a, b;
    ms_step(hv, hw, hj, ion, dt, a, b);
    sm[q.hC] = hm;
    su[q.hC] = a;
    mk[q.hC] = hk;
  }
  __syncthreads();
  if (!m0) {
    at(lv_out, q.g) = T(0);
    at(lw_out, q.g) = T(0);
    return;
  }
  const T nu = mu + dt * apply19(sm, q.C, k18);
  at(grad, q.g) -= static_cast<double>(dt * dB_ds(sm, su, mk, q.C, dq, inv_h2));
  const T dvs_dv = T(1) + dt * (ion.exc * (T(2) * v0 - T(3) * v0 * v0) * w0 * ion.inv_tau_in -
                                ion.inv_tau_out);
  const T dvs_dw = dt * ion.exc * v0 * v0 * (T(1) - v0) * ion.inv_tau_in;
  const T dws_dw = (v0 < ion.v_gate) ? T(1) - dt * ion.inv_tau_open : T(1) - dt * ion.inv_tau_close;
  T lvn = nu * dvs_dv;
  const int cs = at(cross, q.g);
  if ((cs == n || (vprev && cs == n - 1)) && isfinite(at(tstar, q.g))) {
    const T dl = T(2) * (at(tact, q.g) - at(tstar, q.g));
    if (cs == n) lvn += cross_seed(v0, at(vnext, q.g), theta, dt, dl, true);
    else lvn += cross_seed(at(vprev, q.g), v0, theta, dt, dl, false);
  }
  at(lv_out, q.g) = lvn;
  at(lw_out, q.g) = nu * dvs_dw + at(lw_in, q.g) * dws_dw;
}

// loss partials over voxels activated in the run and in the target:
// ((T - T*)^2, count)
template <typename T>
__global__ __launch_bounds__(kBV) void k_loss(int nb, const uint8_t* __restrict__ mask,
                                              const int* __restrict__ cross,
                                              const T* __restrict__ tact,
                                              const T* __restrict__ tstar, double* partials) {
  const int brick = block_brick();
  if (brick >= nb) { idle_partials<2>(partials); return; }
  const int g = brick * kBV + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (mask[g] && cross[g] >= 0 && isfinite(tstar[g])) {
    const double d = static_cast<double>(tact[g]) - static_cast<double>(tstar[g]);
    acc[0] = d * d;
    acc[1] = 1.0;
  }
  block_partials<2>(acc, partials);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_block_max(const LaunchCfg& L, const int* nbr, CoefSet<double> c,
                      double* partials) {
  k_block_max<<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, partials);
}

void launch_scale(const LaunchCfg& L, double* x, const double* y, const double* sums) {
  k_scale<<<L.grid, kBV, 0, L.stream>>>(L.nb, x, y, sums);
}

void launch_tensor_coefs(const LaunchCfg& L, const int* nbr, const uint8_t* mask,
                         const double* fib, const double* scale, double sig_l, double sig_t,
                         double h, double* tens, double* c64[6], float* c32[6],
                         const uint8_t* body, double sig_body) {
  const int64_t stride = (int64_t)(L.nb + 1) * kBV;
  k_tensor<<<L.grid, kBV, 0, L.stream>>>(L.nb, mask, fib, scale, sig_l, sig_t, tens, stride,
                                         body, sig_body);
  CoefOut<double> o64;
  CoefOut<float> o32;
  for (int k = 0; k < 6; ++k) {
    o64.c[k] = c64 ? c64[k] : nullptr;
    o32.c[k] = c32 ? c32[k] : nullptr;
  }
  k_coefs<<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, body ? body : mask, tens, stride,
                                        1.0 / (h * h), o64, o32);
}

void launch_coef_add(const LaunchCfg& L, double* const acc[6], double* const add[6],
                     float* const out32[6]) {
  CoefOut<double> a;
  CoefSet<double> b;
  CoefOut<float> o;
  for (int k = 0; k < 6; ++k) {
    a.c[k] = acc[k];
    b.c[k] = add[k];
    o.c[k] = out32[k];
  }
  k_coef_add<<<L.grid, kBV, 0, L.stream>>>(L.nb, a, b, o);
}

void launch_corner_coefs(const LaunchCfg& L, const int* nbr, const uint8_t* mask,
                         const double* fib, const double* scale, double sig_l, double sig_t,
                         double h, double* tens, double* c64[6], float* c32[6]) {
  const int64_t stride = (int64_t)(L.nb + 1) * kBV;
  k_tensor<<<L.grid, kBV, 0, L.stream>>>(L.nb, mask, fib, scale, sig_l, sig_t, tens, stride,
                                         nullptr, 0.0);
  CoefOut<double> o64;
  CoefOut<float> o32;
  for (int k = 0; k < 6; ++k) {
    o64.c[k] = c64 ? c64[k] : nullptr;
    o32.c[k] = c32 ? c32[k] : nullptr;
  }
  k_coefs27<<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, mask, tens, stride, 1.0 / (16.0 * h * h),
                                          o64, o32);
}

template <typename T>
void launch_unit_tensors(const LaunchCfg& L, const uint8_t* mask, const double* fib,
                         double sig_l, double sig_t, T* out[6]) {
  CoefOut<T> o;
  for (int k = 0; k < 6; ++k) o.c[k] = out[k];
  k_unit_tensor<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, mask, fib, sig_l, sig_t, o);
}

template <typename T>
void launch_explicit(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* v, const T* w,
                     const T* jstim, T* vout, T* wout, T* tact, IonicT<T> ion, T dt, T theta,
                     double tn, int* flags, int* cross, int step) {
  k_explicit<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, v, w, jstim, vout, wout, tact, ion,
                                              dt, theta, tn, flags, cross, step);
}

template <typename T>
void launch_explicit27(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* v, const T* w,
                       const T* jstim, T* vout, T* wout, T* tact, IonicT<T> ion, T dt, T theta,
                       double tn, int* flags) {
  k_explicit27<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, v, w, jstim, vout, wout, tact,
                                                ion, dt, theta, tn, flags);
}

// ---- two-level preconditioner of the bidomain inner solve ----------------
void launch_coarse_setup(const LaunchCfg& L, const int* nbr, double* const ck64[6], double c0,
                         double c1, int n, const int* agg_ptr, const int* agg_brk, const int* agg,
                         double* kb, double* kc) {
  CoefSet<double> c;
  for (int k = 0; k < 6; ++k) c.c[k] = ck64[k];
  k_coarse_brick<<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, c0, c1, kb);
  k_coarse_rows<<<(n + 127) / 128, 128, 0, L.stream>>>(n, agg_ptr, agg_brk, nbr, agg, L.nb, kb,
                                                      kc);
}

void launch_coarse_invert(hipStream_t st, int n, int ld, double* kc, double shift, double* pinv,
                          double* rp, double* cp) {
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int64_t blocks = (nn + 255) / 256;
  k_add_const<<<blocks, 256, 0, st>>>(nn, kc, shift);
  const dim3 tiles((n + 15) / 16, (n + 15) / 16);
  for (int k0 = 0; k0 < n; k0 += kGjPanel) {
    const int bs = std::min(kGjPanel, n - k0);
    k_gj_pivot<<<1, kGjPanel * kGjPanel, 0, st>>>(n, kc, k0, bs, pinv);
    k_gj_panels<<<(static_cast<int64_t>(kGjPanel) * n + 255) / 256, 256, 0, st>>>(n, kc, k0, bs, pinv,
                                                                          rp, cp);
    k_gj_update<<<tiles, 256, 0, st>>>(n, kc, k0, bs, rp, cp);
  }
}

void launch_coarse_pack(hipStream_t st, int n, int ld, const double* kc, double scale,
                        void* kinv) {
  k_to_f16<<<(static_cast<int64_t>(n) * ld + 255) / 256, 256, 0, st>>>(
      n, ld, kc, scale, static_cast<_Float16*>(kinv));
}

void launch_cg2_update(const LaunchCfg& L, float* x, float* r, float* p, float* s, const float* z,
                       const float* w, float* rb, int kind, const CGScalars* cin, CGScalars* cout,
                       const double* prev, unsigned long long* mirror, unsigned seq) {
  k_cg2_update<<<L.pgrid, kBV, 0, L.stream>>>(L.nb, x, r, p, s, z, w, rb, kind, cin, cout, prev,
                                               mirror, seq);
}

void launch_coarse_apply(hipStream_t st, int n, int ld, bool brick_aggs, const int* agg_ptr,
                         const int* agg_brk, const float* rb, float* rc, const void* kinv,
                         float unscale, float* cc, const CGScalars* sc) {
  // single-brick aggregates: the brick sums are the aggregate sums
  if (!brick_aggs) k_agg_sum<<<(n + 127) / 128, 128, 0, st>>>(n, agg_ptr, agg_brk, rb, rc, sc);
  k_coarse_gemv<<<n, 256, 0, st>>>(ld, static_cast<const _Float16*>(kinv), unscale,
                                   brick_aggs ? rb : rc, cc, sc);
}

void launch_cg2_apply(const LaunchCfg& L, const int* nbr, CoefSet<float> c, float c0, float c1,
                      const float* dinv, const float* r, const float* cc, const int* agg, float* z,
                      float* w, const CGScalars* cin, double* parts) {
  k_cg2_apply<<<L.pgrid, kBV, 0, L.stream>>>(L.nb, nbr, c, c0, c1, dinv, r, cc, agg, z, w, cin,
                                              parts, L.rowsn);
}

template <typename T>
void launch_ionic(const LaunchCfg& L, const T* v, const T* w, const T* jstim, T* vs, T* wout,
                  IonicT<T> ion, T dt) {
  k_ionic<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, v, w, jstim, vs, wout, ion, dt);
}

template <typename T>
void launch_be_init(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* v, const T* w,
                    const T* jstim, const T* bprev, const T* qin, T kd, const T* d2,
                    const T* d3, T q2, T q3, T q4, T* bout, T* dout, T* qout, T* x, T* wout,
                    T* z, IonicT<T> ion, T dt, T* tact, T theta, double tprev, int check_prev,
                    int* flags, CGScalars* cout, double* parts, double tol2, int maxit) {
  if constexpr (sizeof(T) == 4) {
    const BeInitArgs A = {v, w, jstim, bprev, qin, d2, d3, bout, dout, qout, x, wout, z,
                          kd, q2, q3, q4, check_prev != 0};
    auto k = L.stream_nt ? k_be_init<true> : k_be_init<false>;
    k<<<L.pgrid, kBV, 0, L.stream>>>(L.nb, nbr, c, A, ion, dt, tact, theta, tprev, flags, cout,
                                     parts, tol2, maxit, L.rowsn);
  } else {
    auto k = L.stream_nt ? k_be_init<T, true> : k_be_init<T, false>;
    k<<<L.pgrid, kBV, 0, L.stream>>>(L.nb, nbr, c, v, w, jstim, bprev, qin, kd, d2, d3, q2, q3,
                                     q4, bout, dout, qout, x, wout, z, ion, dt, tact, theta,
                                     tprev, check_prev, flags, cout, parts, tol2, maxit, L.rowsn);
  }
}


template <typename T>
void launch_pcg_step(const LaunchCfg& L, const int* nbr, CoefSet<T> c, T c0, T c1, T* x,
                     const T* z_in, T* z_out, const T* p_in, T* p_out, const T* t_in, T* t_out,
                     int first, const CGScalars* cin, CGScalars* cout, const double* prev,
                     double* parts, unsigned long long* mirror, unsigned seq) {
  auto k = L.stream_nt ? k_pcg_step<T, true> : k_pcg_step<T, false>;
  k<<<L.pgrid, kBV, 0, L.stream>>>(L.nb, nbr, c, c0, c1, x, z_in, z_out, p_in, p_out, t_in,
                                   t_out, first, cin, cout, prev, parts, L.rowsn, mirror, seq);
}

template <typename T, typename O>
void launch_box_gather(hipStream_t s, const int n[3], int nby, int nbz, const int* brick_id,
                       const T* src, const uint8_t* mask, O* out, O fill) {
  const int64_t N = static_cast<int64_t>(n[0]) * n[1] * n[2];
  const int64_t want = (N + 255) / 256;
  const int blocks = static_cast<int>(want < 8192 ? want : 8192);
  k_box_gather<T, O><<<blocks, 256, 0, s>>>(n[0], n[1], n[2], nby, nbz, brick_id, src, mask, out,
                                            fill);
}
template void launch_box_gather<float, float>(hipStream_t, const int*, int, int, const int*,
                                              const float*, const uint8_t*, float*, float);
template void launch_box_gather<float, double>(hipStream_t, const int*, int, int, const int*,
                                               const float*, const uint8_t*, double*, double);
template void launch_box_gather<double, float>(hipStream_t, const int*, int, int, const int*,
                                               const double*, const uint8_t*, float*, float);
template void launch_box_gather<double, double>(hipStream_t, const int*, int, int, const int*,
                                                const double*, const uint8_t*, double*, double);

template <typename T>
void launch_jacobi(const LaunchCfg& L, const int* nbr, CoefSet<T> c, T dt, const T* dinv,
                   const T* b, const T* x_in, T* x_out) {
  k_jacobi<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, dt, dinv, b, x_in, x_out, L.rowsn);
}

void launch_reduce_sum(hipStream_t s, const double* partials, int nparts, int K, double* out) {
  k_reduce<<<1, kRedThreads, 0, s>>>(partials, nparts, K, out);
}

template <typename T>
void launch_activation(const LaunchCfg& L, const T* vold, const T* vnew, T* tact, T dt, T theta,
                       double tn, int* flags) {
  k_activation<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, vold, vnew, tact, dt, theta, tn, flags);
}

template <typename T>
void launch_dinv(const LaunchCfg& L, const int* nbr, CoefSet<T> c, T c0, T c1, T* dinv) {
  k_dinv<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, c0, c1, dinv);
}

template <typename T>
void launch_sum(const LaunchCfg& L, const T* x, double* partials) {
  k_sum<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, x, partials);
}

template <typename T>
void launch_stim_scatter(hipStream_t s, const int64_t* idx, const double* val, int n, T* jstim,
                         double* qstep) {
  k_stim_scatter<T><<<1, kRedThreads, 0, s>>>(idx, val, n, jstim, qstep);
}

void launch_q_accum(hipStream_t s, double* qacc, const double* qstep, double scale) {
  k_q_accum<<<1, 64, 0, s>>>(qacc, qstep, scale);
}

template <typename T>
void launch_resid64(const LaunchCfg& L, const int* nbr, CoefSet<double> ci, CoefSet<double> ck,
                    const T* vs, const double* phi, double* r64, double* partials) {
  k_resid64<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, ci, ck, vs, phi, r64, partials);
}

void launch_inner_init(const LaunchCfg& L, const double* r64, const uint8_t* mask,
                       const double* sums, double inv_count, float* x, float* r,
                       CGScalars* cout, double* parts, double tol2, int maxit) {
  k_inner_init<<<L.pgrid, kBV, 0, L.stream>>>(L.nb, r64, mask, sums, inv_count, x, r, cout,
                                              parts, tol2, maxit);
}

void launch_phi_correct(const LaunchCfg& L, double* phi, const float* d, const uint8_t* mask,
                        double* partials) {
  k_phi_correct<<<L.grid, kBV, 0, L.stream>>>(L.nb, phi, d, mask, partials);
}

void launch_phi_extrap(const LaunchCfg& L, double* phi, const double* h1, const double* h2,
                       const double* h3, int order) {
  k_phi_extrap<<<L.grid, kBV, 0, L.stream>>>(L.nb, phi, h1, h2, h3, order);
}

void launch_phi_shift(const LaunchCfg& L, double* phi, const uint8_t* mask, const double* sum,
                      double inv_count) {
  k_phi_shift<<<L.grid, kBV, 0, L.stream>>>(L.nb, phi, mask, sum, inv_count);
}

template <typename T>
void launch_parabolic(const LaunchCfg& L, const int* nbr, CoefSet<T> ci, const T* vs,
                      const double* phi, const T* vold, T* vout, T* tact, T dt, T theta,
                      double tn, int* flags) {
  k_parabolic<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, ci, vs, phi, vold, vout, tact, dt,
                                               theta, tn, flags);
}

template <typename T>
void launch_apply(const LaunchCfg& L, const int* nbr, CoefSet<T> c, const T* x, T* y,
                  double* partials) {
  k_apply<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, x, y, partials);
}

template <typename T>
void launch_adj_init(const LaunchCfg& L, const uint8_t* mask, const T* vlast, const T* vprev,
                     const int* cross, const T* tact, const T* tstar, T* lv, T* lw, T dt,
                     T theta, int nlast) {
  k_adj_init<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, mask, vlast, vprev, cross, tact, tstar, lv,
                                              lw, dt, theta, nlast);
}

template <typename T>
void launch_adj_step(const LaunchCfg& L, const int* nbr, CoefSet<T> c, CoefSet<T> d0,
                     const uint8_t* mask, const T* lv_in, const T* lw_in, T* lv_out, T* lw_out,
                     const T* v, const T* w, const T* jstim, const T* vnext, const T* vprev,
                     const int* cross, const T* tact, const T* tstar, double* grad,
                     IonicT<T> ion, T dt, T theta, T inv_h2, int n) {
  k_adj_step<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, nbr, c, d0, mask, lv_in, lw_in, lv_out,
                                              lw_out, v, w, jstim, vnext, vprev, cross, tact,
                                              tstar, grad, ion, dt, theta, inv_h2, n);
}

template <typename T>
void launch_loss(const LaunchCfg& L, const uint8_t* mask, const int* cross, const T* tact,
                 const T* tstar, double* partials) {
  k_loss<T><<<L.grid, kBV, 0, L.stream>>>(L.nb, mask, cross, tact, tstar, partials);
}

#define EP_INST(T)                                                                             \
  template void launch_explicit<T>(const LaunchCfg&, const int*, CoefSet<T>, const T*,         \
                                   const T*, const T*, T*, T*, T*, IonicT<T>, T, T, double,    \
                                   int*, int*, int);                                           \
  template void launch_explicit27<T>(const LaunchCfg&, const int*, CoefSet<T>, const T*,       \
                                     const T*, const T*, T*, T*, T*, IonicT<T>, T, T, double,  \
                                     int*);                                                    \
  template void launch_ionic<T>(const LaunchCfg&, const T*, const T*, const T*, T*, T*,        \
                                IonicT<T>, T);                                                 \
  template void launch_be_init<T>(const LaunchCfg&, const int*, CoefSet<T>, const T*,          \
                                  const T*, const T*, const T*, const T*, T, const T*,         \
                                  const T*, T, T, T, T*, T*, T*, T*, T*, T*, IonicT<T>, T, T*, \
                                  T, double, int, int*, CGScalars*, double*, double, int);     \
  template void launch_pcg_step<T>(const LaunchCfg&, const int*, CoefSet<T>, T, T, T*,        \
                                   const T*, T*, const T*, T*, const T*, T*, int,              \
                                   const CGScalars*, CGScalars*, const double*, double*,       \
                                   unsigned long long*, unsigned);                             \
  template void launch_jacobi<T>(const LaunchCfg&, const int*, CoefSet<T>, T, const T*,       \
                                 const T*, const T*, T*);                                      \
  template void launch_activation<T>(const LaunchCfg&, const T*, const T*, T*, T, T, double,   \
                                     int*);                                                    \
  template void launch_dinv<T>(const LaunchCfg&, const int*, CoefSet<T>, T, T, T*);            \
  template void launch_sum<T>(const LaunchCfg&, const T*, double*);                            \
  template void launch_stim_scatter<T>(hipStream_t, const int64_t*, const double*, int, T*,    \
                                       double*);                                               \
  template void launch_resid64<T>(const LaunchCfg&, const int*, CoefSet<double>,              \
                                  CoefSet<double>, const T*, const double*, double*, double*); \
  template void launch_parabolic<T>(const LaunchCfg&, const int*, CoefSet<T>, const T*,        \
                                    const double*, const T*, T*, T*, T, T, double, int*);      \
  template void launch_apply<T>(const LaunchCfg&, const int*, CoefSet<T>, const T*, T*,        \
                                double*);                                                      \
  template void launch_adj_init<T>(const LaunchCfg&, const uint8_t*, const T*, const T*,       \
                                   const int*, const T*, const T*, T*, T*, T, T, int);         \
  template void launch_adj_step<T>(const LaunchCfg&, const int*, CoefSet<T>, CoefSet<T>,       \
                                   const uint8_t*, const T*, const T*, T*, T*, const T*,       \
                                   const T*, const T*, const T*, const T*, const int*,         \
                                   const T*, const T*, double*, IonicT<T>, T, T, T, int);      \
  template void launch_unit_tensors<T>(const LaunchCfg&, const uint8_t*, const double*, double, \
                                       double, T*[6]);                                         \
  template void launch_loss<T>(const LaunchCfg&, const uint8_t*, const int*, const T*,         \
                               const T*, double*);

EP_INST(float)
EP_INST(double)

}  // namespace ep

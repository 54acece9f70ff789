// Device helpers shared by the per-grid kernels and the batched serving
// kernel: brick/tile indexing, the 19-point operator on an LDS tile, the
// Mitchell-Schaeffer update and block-level partial sums.  See
// ep_internal.h for the data layout.
#pragma once

#include <cmath>
#include <cstdint>

#include "ep_internal.h"

namespace ep {
namespace dev {


__device__ __forceinline__ int tidx(int x, int y, int z) { return (x * kH + y) * kH + z; }

// Element i of a per-voxel array, addressed as base + a 32-bit unsigned
// byte offset: the compiler then keeps the base in scalar registers and
// needs one vector register per distinct index (global_load with saddr)
// instead of a 64-bit address per load.  Every per-voxel array is below
// 4 GiB (the grid creation refuses larger grids), so the offset never wraps.
template <typename T>
__device__ __forceinline__ const T& at(const T* base, int i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     static_cast<uint64_t>(static_cast<uint32_t>(i) *
                                                           static_cast<uint32_t>(sizeof(T))));
}
template <typename T>
__device__ __forceinline__ T& at(T* base, int i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) +
                               static_cast<uint64_t>(static_cast<uint32_t>(i) *
                                                     static_cast<uint32_t>(sizeof(T))));
}

// Workgroups are dealt round-robin to the 8 XCDs; hand each XCD a contiguous
// run of bricks so that halo neighbours tend to sit in the same L2.
__device__ __forceinline__ int block_brick() {
  const int per = gridDim.x / kXcd;
  const int b = blockIdx.x;
  return (b % kXcd) * per + b / kXcd;
}

// Halo cell k in [0, 480): 6 faces x 64 cells, then 12 edges x 8 cells.
// Coordinates are tile coordinates in [0, 10) (0 and 9 are the halo).
__device__ __forceinline__ void halo_cell(int k, int& hx, int& hy, int& hz) {
  if (k < 384) {
    const int f = k >> 6, m = k & 63;
    const int d = f >> 1, side = (f & 1) ? 9 : 0;
    const int i = (m >> 3) + 1, j = (m & 7) + 1;
    if (d == 0) { hx = side; hy = i; hz = j; }
    else if (d == 1) { hx = i; hy = side; hz = j; }
    else { hx = i; hy = j; hz = side; }
  } else {
    const int k2 = k - 384;
    const int e = k2 >> 3, t = (k2 & 7) + 1;
    const int pair = e >> 2;
    const int s1 = (e & 2) ? 9 : 0, s2 = (e & 1) ? 9 : 0;
    if (pair == 0) { hx = s1; hy = s2; hz = t; }
    else if (pair == 1) { hx = s1; hy = t; hz = s2; }
    else { hx = t; hy = s1; hz = s2; }
  }
}

// global index of tile cell (hx, hy, hz) of the brick whose neighbour row is nbs
__device__ __forceinline__ int tile_global(const int* nbs, int hx, int hy, int hz) {
  const int ox = (hx == 0) ? 0 : (hx == 9 ? 2 : 1);
  const int oy = (hy == 0) ? 0 : (hy == 9 ? 2 : 1);
  const int oz = (hz == 0) ? 0 : (hz == 9 ? 2 : 1);
  const int bk = nbs[ox * 9 + oy * 3 + oz];
  return bk * kBV + ((((hx + 7) & 7) * 8 + ((hy + 7) & 7)) * 8 + ((hz + 7) & 7));
}

// global index of voxel (lx+dx, ly+dy, lz+dz), d in {-1, 0, 1}
__device__ __forceinline__ int nb_global(const int* nbs, int brick, int lx, int ly, int lz,
                                         int dx, int dy, int dz) {
  const int tx = lx + dx, ty = ly + dy, tz = lz + dz;
  const int ox = tx < 0 ? 0 : (tx > 7 ? 2 : 1);
  const int oy = ty < 0 ? 0 : (ty > 7 ? 2 : 1);
  const int oz = tz < 0 ? 0 : (tz > 7 ? 2 : 1);
  const int slot = ox * 9 + oy * 3 + oz;
  const int bk = (slot == 13) ? brick : nbs[slot];
  return bk * kBV + (((tx & 7) * 8 + (ty & 7)) * 8 + (tz & 7));
}

// Row liveness.  A brick row is the 8 voxels (lx, ly, 0..7), 32 contiguous
// bytes in FP32; bit lx*8 + ly of a brick's row mask is set when the row
// holds tissue.  rowm[27] holds the masks of a brick's 3x3x3 neighbourhood
// (same slots as nbs).  A voxel of an empty row carries nothing the
// operator uses (its weights are zero, and the kernels that skip rows never
// store there), so its loads are redirected to the same offset in the ghost
// brick, which is all zeros and stays in L2: the loads remain unconditional
// (no branch, no wait) and the row's HBM traffic disappears.
__device__ __forceinline__ bool vox_live(const uint64_t* rowm, int tx, int ty, int tz) {
  const int ox = tx < 0 ? 0 : (tx > 7 ? 2 : 1);
  const int oy = ty < 0 ? 0 : (ty > 7 ? 2 : 1);
  const int oz = tz < 0 ? 0 : (tz > 7 ? 2 : 1);
  return (rowm[ox * 9 + oy * 3 + oz] >> ((((tx & 7) << 3) | (ty & 7)))) & 1;
}

// The 18 off-centre weights of voxel p of the 19-point operator, in the order
//  0 ax(p)   1 ax(p-x)  2 ay(p)   3 ay(p-y)  4 az(p)   5 az(p-z)
//  6 bxy(p)  7 bxy(p-x-y)  8 bxy(p-y)  9 bxy(p-x)
// 10 bxz(p) 11 bxz(p-x-z) 12 bxz(p-z) 13 bxz(p-x)
// 14 byz(p) 15 byz(p-y-z) 16 byz(p-z) 17 byz(p-y)
// With rowm, a weight stored in an empty row is loaded from the ghost brick
// (nb is the ghost brick id), so it reads zero.  ld(p, i) loads element i of
// array p (at() unless a caller needs another access form).
struct AtLoad {
  template <typename T>
  __device__ __forceinline__ T operator()(const T* p, int i) const { return at(p, i); }
};

template <typename T, typename Ld = AtLoad>
__device__ __forceinline__ void gather18(const CoefSet<T>& c, const int* nbs, int brick, int lx,
                                         int ly, int lz, T k[18],
                                         const uint64_t* rowm = nullptr, int nb = 0,
                                         Ld ld = Ld{}) {
  int g = brick * kBV + (lx * 8 + ly) * 8 + lz;
  int gx = nb_global(nbs, brick, lx, ly, lz, -1, 0, 0);
  int gy = nb_global(nbs, brick, lx, ly, lz, 0, -1, 0);
  int gz = nb_global(nbs, brick, lx, ly, lz, 0, 0, -1);
  int gxy = nb_global(nbs, brick, lx, ly, lz, -1, -1, 0);
  int gxz = nb_global(nbs, brick, lx, ly, lz, -1, 0, -1);
  int gyz = nb_global(nbs, brick, lx, ly, lz, 0, -1, -1);
  if (rowm) {
    const int gh = nb * kBV + (lx * 8 + ly) * 8 + lz;
    const bool l0 = vox_live(rowm, lx, ly, lz);
    g = l0 ? g : gh;
    gx = (l0 && vox_live(rowm, lx - 1, ly, lz)) ? gx : gh;
    gy = (l0 && vox_live(rowm, lx, ly - 1, lz)) ? gy : gh;
    gz = (l0 && vox_live(rowm, lx, ly, lz - 1)) ? gz : gh;
    gxy = (l0 && vox_live(rowm, lx - 1, ly - 1, lz)) ? gxy : gh;
    gxz = (l0 && vox_live(rowm, lx - 1, ly, lz - 1)) ? gxz : gh;
    gyz = (l0 && vox_live(rowm, lx, ly - 1, lz - 1)) ? gyz : gh;
  }
  k[0] = ld(c.c[CX], g);
  k[1] = ld(c.c[CX], gx);
  k[2] = ld(c.c[CY], g);
  k[3] = ld(c.c[CY], gy);
  k[4] = ld(c.c[CZ], g);
  k[5] = ld(c.c[CZ], gz);
  k[6] = ld(c.c[CXY], g);
  k[7] = ld(c.c[CXY], gxy);
  k[8] = ld(c.c[CXY], gy);
  k[9] = ld(c.c[CXY], gx);
  k[10] = ld(c.c[CXZ], g);
  k[11] = ld(c.c[CXZ], gxz);
  k[12] = ld(c.c[CXZ], gz);
  k[13] = ld(c.c[CXZ], gx);
  k[14] = ld(c.c[CYZ], g);
  k[15] = ld(c.c[CYZ], gyz);
  k[16] = ld(c.c[CYZ], gz);
  k[17] = ld(c.c[CYZ], gy);
}

// (A u)_p from the LDS tile s at tile cell C.  Faces: a (u_q - u_p).  Each
// 2x2 block in plane (d, d') couples p with its diagonal partner: +b along
// (+d,+d') / (-d,-d') and -b along (+d,-d') / (-d,+d').
template <typename T>
__device__ __forceinline__ T apply19(const T* s, int C, const T k[18]) {
  const T u = s[C];
  T a = k[0] * (s[C + 100] - u) + k[1] * (s[C - 100] - u) + k[2] * (s[C + 10] - u) +
        k[3] * (s[C - 10] - u) + k[4] * (s[C + 1] - u) + k[5] * (s[C - 1] - u);
  a += k[6] * (s[C + 110] - u) + k[7] * (s[C - 110] - u) - k[8] * (s[C + 90] - u) -
       k[9] * (s[C - 90] - u);
  a += k[10] * (s[C + 101] - u) + k[11] * (s[C - 101] - u) - k[12] * (s[C + 99] - u) -
       k[13] * (s[C - 99] - u);
  a += k[14] * (s[C + 11] - u) + k[15] * (s[C - 11] - u) - k[16] * (s[C + 9] - u) -
       k[17] * (s[C - 9] - u);
  return a;
}

template <typename T>
__device__ __forceinline__ T diag19(const T k[18]) {
  return -(k[0] + k[1] + k[2] + k[3] + k[4] + k[5]) - (k[6] + k[7]) + (k[8] + k[9]) -
         (k[10] + k[11]) + (k[12] + k[13]) - (k[14] + k[15]) + (k[16] + k[17]);
}

// One explicit Euler step of Mitchell-Schaeffer; the gate branch is decided
// on the pre-step v and taken as a select.
template <typename T>
__device__ __forceinline__ void ms_step(T v, T w, T js, const IonicT<T>& p, T dt, T& vs,
                                        T& ws) {
  const T jin = p.exc * v * v * (T(1) - v) * w * p.inv_tau_in;
  const T jout = -v * p.inv_tau_out;
  const T dw = (v < p.v_gate) ? (T(1) - w) * p.inv_tau_open : -w * p.inv_tau_close;
  vs = v + dt * (jin + jout + js);
  ws = w + dt * dw;
}

// Sum K per-thread doubles over the block; thread k < K writes slot k.
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* partials) {
  __shared__ double red[K][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    partials[threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

template <int K>
__device__ __forceinline__ void idle_partials(double* partials) {
  if (partials && threadIdx.x < K) partials[threadIdx.x * gridDim.x + blockIdx.x] = 0.0;
}

// Common prologue of the stencil kernels: the thread's own voxel, its halo
// cell (threads < 480) and their tile cells.
// With rowm (and the ghost brick id nb), live tells whether the own voxel
// lies in a row holding tissue; gl / hgl are the indices to load the own
// voxel / the halo cell from: the real ones for live rows, the same offset
// in the ghost brick otherwise.  Without rowm, gl = g, hgl = hg, live = true.
struct Cell {
  int lx, ly, lz, g, C;     // own voxel
  bool has_halo;
  int hg, hC;               // halo cell: global index and tile cell
  bool live;
  int gl, hgl;
};

__device__ __forceinline__ Cell cell_setup(const int* nbs, int brick,
                                           const uint64_t* rowm = nullptr, int nb = 0) {
  Cell c;
  const int t = threadIdx.x;
  c.lx = t >> 6;
  c.ly = (t >> 3) & 7;
  c.lz = t & 7;
  c.g = brick * kBV + t;
  c.C = tidx(c.lx + 1, c.ly + 1, c.lz + 1);
  c.has_halo = t < kHalo;
  c.hg = 0;
  c.hC = 0;
  c.live = rowm ? vox_live(rowm, c.lx, c.ly, c.lz) : true;
  c.gl = c.live ? c.g : nb * kBV + t;
  c.hgl = 0;
  if (c.has_halo) {
    int hx, hy, hz;
    halo_cell(t, hx, hy, hz);
    c.hg = tile_global(nbs, hx, hy, hz);
    c.hC = tidx(hx, hy, hz);
    c.hgl = (!rowm || vox_live(rowm, hx - 1, hy - 1, hz - 1)) ? c.hg : nb * kBV + t;
  }
  return c;
}

// ---------------------------------------------------------------------------
// Staging a brick into LDS with direct global-to-LDS loads (the pipelined
// brick loops): the weight halo (the weights of cells on a brick's -x, -y,
// -z sides that its own voxels' 19-point rows use) and helpers.
// Weight halo: CX on the x = -1 plane (y*8+z), CY on y = -1 (x*8+z), CZ on
// z = -1 (x*8+y); then 136 entries for each edge weight:
//   CXY: x = -1 plane (y*8+z), y = -1 plane (x*8+z), the (-1,-1,z) edge;
//   CXZ: x = -1 (y*8+z), z = -1 (x*8+y), the (-1,y,-1) edge;
//   CYZ: y = -1 (x*8+z), z = -1 (x*8+y), the (x,-1,-1) edge.
constexpr int kWHalo = 600;
constexpr int kWhCX = 0, kWhCY = 64, kWhCZ = 128, kWhCXY = 192, kWhCXZ = 328, kWhCYZ = 464;
// entry m of weight array a's halo: coordinates relative to the brick
__device__ __forceinline__ void wh_coords(int a, int m, int& tx, int& ty, int& tz) {
  const int i = (m >> 3) & 7, j = m & 7, e = m - 128;
  switch (a) {
    case CX: tx = -1; ty = i; tz = j; break;
    case CY: tx = i; ty = -1; tz = j; break;
    case CZ: tx = i; ty = j; tz = -1; break;
    case CXY:
      if (m < 64) { tx = -1; ty = i; tz = j; }
      else if (m < 128) { tx = i; ty = -1; tz = j; }
      else { tx = -1; ty = -1; tz = e; }
      break;
    case CXZ:
      if (m < 64) { tx = -1; ty = i; tz = j; }
      else if (m < 128) { tx = i; ty = j; tz = -1; }
      else { tx = -1; ty = e; tz = -1; }
      break;
    default:   // CYZ
      if (m < 64) { tx = i; ty = -1; tz = j; }
      else if (m < 128) { tx = i; ty = j; tz = -1; }
      else { tx = e; ty = -1; tz = -1; }
  }
}

// gather18's weights from a staged brick F (flat stage): the own cells of
// the six weight arrays at W (array a at W + a * 512), the weight halo at H
template <int W, int H>
__device__ __forceinline__ void gather18_lds(const float* F, int t, int lx, int ly, int lz,
                                             float k[18]) {
  k[0] = F[W + CX * kBV + t];
  k[1] = F[lx ? W + CX * kBV + t - 64 : H + kWhCX + ly * 8 + lz];
  k[2] = F[W + CY * kBV + t];
  k[3] = F[ly ? W + CY * kBV + t - 8 : H + kWhCY + lx * 8 + lz];
  k[4] = F[W + CZ * kBV + t];
  k[5] = F[lz ? W + CZ * kBV + t - 1 : H + kWhCZ + lx * 8 + ly];
  k[6] = F[W + CXY * kBV + t];
  k[7] = F[(lx && ly) ? W + CXY * kBV + t - 72
           : (!lx && !ly) ? H + kWhCXY + 128 + lz
           : !lx ? H + kWhCXY + (ly - 1) * 8 + lz : H + kWhCXY + 64 + (lx - 1) * 8 + lz];
  k[8] = F[ly ? W + CXY * kBV + t - 8 : H + kWhCXY + 64 + lx * 8 + lz];
  k[9] = F[lx ? W + CXY * kBV + t - 64 : H + kWhCXY + ly * 8 + lz];
  k[10] = F[W + CXZ * kBV + t];
  k[11] = F[(lx && lz) ? W + CXZ * kBV + t - 65
            : (!lx && !lz) ? H + kWhCXZ + 128 + ly
            : !lx ? H + kWhCXZ + ly * 8 + (lz - 1) : H + kWhCXZ + 64 + (lx - 1) * 8 + ly];
  k[12] = F[lz ? W + CXZ * kBV + t - 1 : H + kWhCXZ + 64 + lx * 8 + ly];
  k[13] = F[lx ? W + CXZ * kBV + t - 64 : H + kWhCXZ + ly * 8 + lz];
  k[14] = F[W + CYZ * kBV + t];
  k[15] = F[(ly && lz) ? W + CYZ * kBV + t - 9
            : (!ly && !lz) ? H + kWhCYZ + 128 + lx
            : !ly ? H + kWhCYZ + lx * 8 + (lz - 1) : H + kWhCYZ + 64 + lx * 8 + (ly - 1)];
  k[16] = F[lz ? W + CYZ * kBV + t - 1 : H + kWhCYZ + 64 + lx * 8 + ly];
  k[17] = F[ly ? W + CYZ * kBV + t - 8 : H + kWhCYZ + lx * 8 + lz];
}

// one direct global-to-LDS dword load per active lane: lane i of the wave
// writes dst[i] (dst the same in every lane of the wave)
template <bool NT>
__device__ __forceinline__ void lds_load(const float* base, int i, float* dst) {
  const float* src = reinterpret_cast<const float*>(
      reinterpret_cast<const char*>(base) +
      static_cast<uint64_t>(static_cast<uint32_t>(i) * 4u));
  __builtin_amdgcn_global_load_lds(src, dst, 4, 0, NT ? 2 : 0);
}

// weight-halo entries [m0, m0 + n) of array a, one per lane from lane l0 on
__device__ __forceinline__ void wh_load(float* F, const float* base, int a, int m0, int off,
                                        int lane, int l0, int n, int nb, const int* nbs,
                                        const uint64_t* rowm) {
  if (lane < l0 || lane >= l0 + n) return;
  const int m = m0 + lane - l0;
  int tx, ty, tz;
  wh_coords(a, m, tx, ty, tz);
  const int ox = tx < 0 ? 0 : 1, oy = ty < 0 ? 0 : 1, oz = tz < 0 ? 0 : 1;
  const int g = vox_live(rowm, tx, ty, tz)
                    ? nbs[ox * 9 + oy * 3 + oz] * kBV + (((tx & 7) * 8 + (ty & 7)) * 8 + (tz & 7))
                    : nb * kBV + lane;
  lds_load<false>(base, g, F + off + m0 - l0);
}

// global index a halo thread t (< 480) loads: its halo cell, or the ghost
// brick when the cell's row holds no tissue
__device__ __forceinline__ int halo_index(int t, int nb, const int* nbs, const uint64_t* rowm) {
  int hx, hy, hz;
  halo_cell(t, hx, hy, hz);
  return vox_live(rowm, hx - 1, hy - 1, hz - 1) ? tile_global(nbs, hx, hy, hz) : nb * kBV + t;
}

// stage the six weight arrays of a brick: own cells (index gl) at W, the
// weight halo at H, one array per wave (wave-uniform bases)
template <int W, int H>
__device__ __forceinline__ void stage_weights(float* F, int gl, int nb, const int* nbs,
                                              const uint64_t* rowm, const CoefSet<float>& c) {
  const int t = threadIdx.x, w0 = t & ~63, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int a = 0; a < 6; ++a) lds_load<false>(c.c[a], gl, F + W + a * kBV + w0);
  switch (wave) {
    case 0:
      wh_load(F, c.c[CX], CX, 0, H + kWhCX, lane, 0, 64, nb, nbs, rowm);
      wh_load(F, c.c[CYZ], CYZ, 64, H + kWhCYZ, lane, 0, 64, nb, nbs, rowm);
      break;
    case 1:
      wh_load(F, c.c[CY], CY, 0, H + kWhCY, lane, 0, 64, nb, nbs, rowm);
      wh_load(F, c.c[CXY], CXY, 128, H + kWhCXY, lane, 0, 8, nb, nbs, rowm);
      wh_load(F, c.c[CXZ], CXZ, 128, H + kWhCXZ, lane, 8, 8, nb, nbs, rowm);
      wh_load(F, c.c[CYZ], CYZ, 128, H + kWhCYZ, lane, 16, 8, nb, nbs, rowm);
      break;
    case 2: wh_load(F, c.c[CZ], CZ, 0, H + kWhCZ, lane, 0, 64, nb, nbs, rowm); break;
    case 3: wh_load(F, c.c[CXY], CXY, 0, H + kWhCXY, lane, 0, 64, nb, nbs, rowm); break;
    case 4: wh_load(F, c.c[CXY], CXY, 64, H + kWhCXY, lane, 0, 64, nb, nbs, rowm); break;
    case 5: wh_load(F, c.c[CXZ], CXZ, 0, H + kWhCXZ, lane, 0, 64, nb, nbs, rowm); break;
    case 6: wh_load(F, c.c[CXZ], CXZ, 64, H + kWhCXZ, lane, 0, 64, nb, nbs, rowm); break;
    default: wh_load(F, c.c[CYZ], CYZ, 0, H + kWhCYZ, lane, 0, 64, nb, nbs, rowm);
  }
}

}  // namespace dev
}  // namespace ep

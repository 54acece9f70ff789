/*
 * ep_oracle.c -- plain FP64 CPU reference ("the oracle") for the
 * operator-split, matrix-free finite-volume monodomain / bidomain voxel step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library
 * shares no code, header, table or helper with it; both consume the same
 * seeded problem instances and nothing else.
 *
 * Everything is double precision, written for clarity, not speed: each
 * function follows the definition it cites, with no blocking or fusion.
 *
 * Model (thesis, Cardiac Multiphysics chapter, Electrophysiology section;
 * Algorithm Details chapter, Electrophysiology section):
 *   - Mitchell-Schaeffer ionic model, eqn:ms1 / eqn:ms2, integrated by one
 *     explicit Euler step per time step (Reaction subsection).  Readings: the
 *     gate relaxes as -w/tau_close above v_gate (the printed (1-w)/tau_close
 *     never repolarises, contradicting the figure of the action potential and
 *     the cited original model) and the w update starts from w, not v.
 *   - Conductivity tensor per voxel, eqn:sigma1: D = s*(sT I + (sL-sT) f f^T)
 *     with an optional per-voxel scale s.
 *   - Diffusion operator A: the symmetric 19-point finite-volume operator in
 *     energy form (definition below).  For isotropic D it is exactly the
 *     cell-centred 7-point Neumann Laplacian.  Face tensors are the mean of
 *     the two voxel tensors, edge tensors the mean of the four voxel tensors
 *     of the 2x2 block (the thesis interpolates the conductivity to the
 *     gradient points, Algorithm Details chapter, Diffusion subsection).
 *   - Monodomain (eqn:monodomain1, chi_m*C_m = 1, lambda/(1+lambda) folded
 *     into D): v_{n+1} = v* + dt A v* (explicit) or (I - dt A) v_{n+1} = v*
 *     (implicit Euler: Linear Solver section, "Implicit Euler"), solved here
 *     by Jacobi-preconditioned CG to a tolerance, or by the thesis's own fixed
 *     number of Jacobi sweeps (eqn:iejac1).
 *   - Bidomain (eqn:bidomain1, v_i = v + phi_e):
 *     -(A_i + A_e) phi = A_i v*, sum_tissue phi = 0;  v_{n+1} = v* + dt A_i(v* + phi),
 *     optionally with a conducting bath around the heart for the ECG
 *     (orc_solve_elliptic), and the six limb leads (orc_ecg).
 *   - Optionally (diff 3, monodomain, explicit only) the thesis's own
 *     corner-gradient operator A27 (orc_apply27), for comparison.
 *   - Activation time: first step with v_n < theta <= v_{n+1}; linear
 *     interpolation T = t_n + dt (theta - v_n)/(v_{n+1} - v_n).
 *
 * Energy definition of A (tissue set T, h = voxel width):
 *   E(v) = sum over faces f=(p,p+e_d), p,q in T:       Df_dd (v_q - v_p)^2 / h^2
 *        + sum over 2x2 blocks in plane (d,d'), d<d', all four voxels in T:
 *                                                       2 De_dd' g_d g_d'
 *   g_d  = (v[+d] + v[+d+d'] - v[0] - v[+d']) / (2h)  (block-centred gradient,
 *          the thesis's reference gradient at a volume centre, eqn:refgrad2)
 *   (A v)_p = -1/2 dE/dv_p.
 *
 * Index convention: flat index (x*ny + y)*nz + z, z fastest.
 * Tensor storage: D[c*N + p], c = 0..5 for xx, yy, zz, xy, xz, yz.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_XX 0
#define ORC_YY 1
#define ORC_ZZ 2
#define ORC_XY 3
#define ORC_XZ 4
#define ORC_YZ 5

typedef struct {
  int32_t lo[3], hi[3];
  double center[3];
  double radius;
  double amp, t_on, t_off;
} orc_stim;

typedef struct {
  int32_t n[3];
  double h, dt, theta;
  double tau_in, tau_out, tau_open, tau_close, v_gate, exc;
  int32_t model;      /* 0 monodomain, 1 bidomain */
  int32_t diff;       /* 0 explicit, 1 implicit Euler by PCG, 2 implicit Euler
                         by a fixed number of Jacobi sweeps (monodomain),
                         3 explicit with the corner-gradient operator A27
                         (monodomain) */
  double cg_rtol;
  int32_t cg_maxit;
  int32_t n_stim;
  const orc_stim* stim;
  const uint8_t* mask;
  const double* Di;   /* 6*N voxel tensors (monodomain D, or intracellular) */
  const double* De;   /* 6*N extracellular tensors (bidomain) */
  int32_t jacobi_sweeps;  /* diff 2: sweeps per step */
  const uint8_t* bath;    /* bidomain: NULL, or 1 on conducting body-tissue
                             (bath / torso) voxels outside the heart */
  double sig_bath;        /* isotropic bath conductivity */
} orc_problem;

typedef struct {
  double* v;
  double* w;
  double* phi;
  double* tact;
  int64_t step;
} orc_state;

typedef struct {
  int64_t cg_iters;   /* total CG iterations in the call */
  int32_t cg_max;     /* largest iteration count of one solve */
  int32_t cg_fail;    /* solves that hit the iteration limit */
  double q_stim;      /* dt * h^3 * sum J_stim accumulated over the call */
  double mass;        /* h^3 * sum_tissue v at the end of the call */
} orc_info;

static inline int64_t idx3(const int32_t n[3], int x, int y, int z) {
  return ((int64_t)x * n[1] + y) * n[2] + z;
}

static inline int inside(const int32_t n[3], int x, int y, int z) {
  return x >= 0 && y >= 0 && z >= 0 && x < n[0] && y < n[1] && z < n[2];
}

static inline int64_t nvox(const int32_t n[3]) {
  return (int64_t)n[0] * n[1] * n[2];
}

/* component index of the off-diagonal tensor entry for axes d < e */
static inline int offdiag(int d, int e) {
  if (d == 0 && e == 1) return ORC_XY;
  if (d == 0 && e == 2) return ORC_XZ;
  return ORC_YZ;
}

/* ------------------------------------------------------------------------ */
/* conductivity tensors, eqn:sigma1                                          */
/* ------------------------------------------------------------------------ */
void orc_tensors(const int32_t n[3], const uint8_t* mask, const double* fib,
                 const double* scale, double sig_l, double sig_t, double* D) {
  const int64_t N = nvox(n);
  for (int64_t p = 0; p < N; ++p) {
    const double s = scale ? scale[p] : 1.0;
    const double f0 = fib[3 * p], f1 = fib[3 * p + 1], f2 = fib[3 * p + 2];
    const double a = sig_l - sig_t;
    const int t = mask[p] != 0;
    D[ORC_XX * N + p] = t ? s * (sig_t + a * f0 * f0) : 0.0;
    D[ORC_YY * N + p] = t ? s * (sig_t + a * f1 * f1) : 0.0;
    D[ORC_ZZ * N + p] = t ? s * (sig_t + a * f2 * f2) : 0.0;
    D[ORC_XY * N + p] = t ? s * (a * f0 * f1) : 0.0;
    D[ORC_XZ * N + p] = t ? s * (a * f0 * f2) : 0.0;
    D[ORC_YZ * N + p] = t ? s * (a * f1 * f2) : 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* the diffusion operator, (A v)_p = -1/2 dE/dv_p                            */
/* ------------------------------------------------------------------------ */

/* Face (p, p+e_d) contributes Df (v_q - v_p)^2 / h^2 to E; its share of
 * -1/2 dE/dv_p is Df (v_q - v_p) / h^2 for either end p.
 * A 2x2 block with lower corner b in plane (d,e) contributes
 * 2 De g_d g_e; with p = b + a_d e_d + a_e e_e (a in {0,1}),
 * dg_d/dv_p = (a_d ? +1 : -1)/(2h) and dg_e/dv_p = (a_e ? +1 : -1)/(2h), so
 * its share of -1/2 dE/dv_p is -De (dg_d/dv_p g_e + g_d dg_e/dv_p). */
static double apply_at(const int32_t n[3], double h, const uint8_t* mask,
                       const double* D, const double* v, int x, int y, int z) {
  const int64_t N = nvox(n);
  const int64_t p = idx3(n, x, y, z);
  if (!mask[p]) return 0.0;
  const int c[3] = {x, y, z};
  double acc = 0.0;
  /* faces */
  for (int d = 0; d < 3; ++d) {
    for (int s = -1; s <= 1; s += 2) {
      int q3[3] = {c[0], c[1], c[2]};
      q3[d] += s;
      if (!inside(n, q3[0], q3[1], q3[2])) continue;
      const int64_t q = idx3(n, q3[0], q3[1], q3[2]);
      if (!mask[q]) continue;
      const double Df = 0.5 * (D[d * N + p] + D[d * N + q]);
      acc += Df * (v[q] - v[p]) / (h * h);
    }
  }
  /* edge blocks */
  for (int d = 0; d < 3; ++d) {
    for (int e = d + 1; e < 3; ++e) {
      const int comp = offdiag(d, e);
      for (int ad = 0; ad <= 1; ++ad) {
        for (int ae = 0; ae <= 1; ++ae) {
          int b[3] = {c[0], c[1], c[2]};
          b[d] -= ad;
          b[e] -= ae;
          /* the four corners b, b+e_d, b+e_e, b+e_d+e_e */
          int64_t k[2][2];
          int ok = 1;
          for (int i = 0; i <= 1 && ok; ++i) {
            for (int j = 0; j <= 1 && ok; ++j) {
              int q3[3] = {b[0], b[1], b[2]};
              q3[d] += i;
              q3[e] += j;
              if (!inside(n, q3[0], q3[1], q3[2])) { ok = 0; break; }
              k[i][j] = idx3(n, q3[0], q3[1], q3[2]);
              if (!mask[k[i][j]]) ok = 0;
            }
          }
          if (!ok) continue;
          const double De = 0.25 * (D[comp * N + k[0][0]] + D[comp * N + k[1][0]] +
                                    D[comp * N + k[0][1]] + D[comp * N + k[1][1]]);
          const double gd = (v[k[1][0]] + v[k[1][1]] - v[k[0][0]] - v[k[0][1]]) / (2.0 * h);
          const double ge = (v[k[0][1]] + v[k[1][1]] - v[k[0][0]] - v[k[1][0]]) / (2.0 * h);
          const double dgd = (ad ? 1.0 : -1.0) / (2.0 * h);
          const double dge = (ae ? 1.0 : -1.0) / (2.0 * h);
          acc += -De * (dgd * ge + gd * dge);
        }
      }
    }
  }
  return acc;
}

void orc_apply(const int32_t n[3], double h, const uint8_t* mask, const double* D,
               const double* v, double* out) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n[0]; ++x)
    for (int y = 0; y < n[1]; ++y)
      for (int z = 0; z < n[2]; ++z)
        out[idx3(n, x, y, z)] = apply_at(n, h, mask, D, v, x, y, z);
}

/* A_pp = -1/2 d^2E/dv_p^2: each face gives -Df/h^2; each block gives
 * -De * 2 (dg_d/dv_p)(dg_e/dv_p). */
void orc_diag(const int32_t n[3], double h, const uint8_t* mask, const double* D,
              double* diag) {
  const int64_t N = nvox(n);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n[0]; ++x)
    for (int y = 0; y < n[1]; ++y)
      for (int z = 0; z < n[2]; ++z) {
        const int64_t p = idx3(n, x, y, z);
        double acc = 0.0;
        if (mask[p]) {
          const int c[3] = {x, y, z};
          for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
              int q3[3] = {c[0], c[1], c[2]};
              q3[d] += s;
              if (!inside(n, q3[0], q3[1], q3[2])) continue;
              const int64_t q = idx3(n, q3[0], q3[1], q3[2]);
              if (!mask[q]) continue;
              acc -= 0.5 * (D[d * N + p] + D[d * N + q]) / (h * h);
            }
          for (int d = 0; d < 3; ++d)
            for (int e = d + 1; e < 3; ++e) {
              const int comp = offdiag(d, e);
              for (int ad = 0; ad <= 1; ++ad)
                for (int ae = 0; ae <= 1; ++ae) {
                  int b[3] = {c[0], c[1], c[2]};
                  b[d] -= ad;
                  b[e] -= ae;
                  double sum = 0.0;
                  int ok = 1;
                  for (int i = 0; i <= 1 && ok; ++i)
                    for (int j = 0; j <= 1 && ok; ++j) {
                      int q3[3] = {b[0], b[1], b[2]};
                      q3[d] += i;
                      q3[e] += j;
                      if (!inside(n, q3[0], q3[1], q3[2])) { ok = 0; break; }
                      const int64_t q = idx3(n, q3[0], q3[1], q3[2]);
                      if (!mask[q]) { ok = 0; break; }
                      sum += D[comp * N + q];
                    }
                  if (!ok) continue;
                  const double De = 0.25 * sum;
                  const double dgd = (ad ? 1.0 : -1.0) / (2.0 * h);
                  const double dge = (ae ? 1.0 : -1.0) / (2.0 * h);
                  acc -= De * 2.0 * dgd * dge;
                }
            }
        }
        diag[p] = acc;
      }
}

/* ------------------------------------------------------------------------ */
/* the thesis's corner-gradient operator (Matrix-Free Assembly section,     */
/* eqn:ass1 - eqn:ass3; Algorithm Details chapter, Diffusion subsection)    */
/* ------------------------------------------------------------------------ */

/* (A27 v)_p from the 27 values around p, taken through the thesis's chain of
 * small matrices in order:
 *   D1  reference gradient at each of the 8 corners of p's volume, from the
 *       2x2x2 block of voxels meeting at that corner: per axis, the mean of
 *       the block's four differences along it (unit reference spacing);
 *   S1  the conductivity tensor at the corner: the mean of the block's eight
 *       voxel tensors (the thesis interpolates the fibre field to the
 *       gradient points; averaging tensors keeps f and -f equivalent);
 *   F1  inverse deformation gradient: I/h on the undeformed grid;
 *   D2  the flux at each face midpoint: the mean over the face's 4 corners;
 *   F2 N1  outward unit normal dotted with each face flux, summed over the 6
 *       faces, times face area over volume (1/h undeformed).
 * Reading (no flux): a corner whose block leaves the grid or holds a
 * non-tissue voxel carries no flux. */
static double apply27_at(const int32_t n[3], double h, const uint8_t* mask,
                         const double* D, const double* v, int x, int y, int z) {
  const int64_t N = nvox(n);
  const int64_t p = idx3(n, x, y, z);
  if (!mask[p]) return 0.0;
  double face[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};   /* [axis][- side, + side] */
  for (int a = 0; a <= 1; ++a)
    for (int b = 0; b <= 1; ++b)
      for (int c = 0; c <= 1; ++c) {
        /* corner at p + (a - 1/2, b - 1/2, c - 1/2) h; its block's lowest voxel */
        const int bx = x + a - 1, by = y + b - 1, bz = z + c - 1;
        double val[2][2][2];
        double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int ok = 1;
        for (int i = 0; i <= 1 && ok; ++i)
          for (int j = 0; j <= 1 && ok; ++j)
            for (int k = 0; k <= 1 && ok; ++k) {
              if (!inside(n, bx + i, by + j, bz + k)) { ok = 0; break; }
              const int64_t q = idx3(n, bx + i, by + j, bz + k);
              if (!mask[q]) { ok = 0; break; }
              val[i][j][k] = v[q];
              for (int m = 0; m < 6; ++m) S[m] += D[m * N + q] / 8.0;
            }
        if (!ok) continue;
        /* D1 */
        double gr[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j <= 1; ++j)
          for (int k = 0; k <= 1; ++k) {
            gr[0] += 0.25 * (val[1][j][k] - val[0][j][k]);
            gr[1] += 0.25 * (val[j][1][k] - val[j][0][k]);
            gr[2] += 0.25 * (val[j][k][1] - val[j][k][0]);
          }
        /* S1 */
        const double fl[3] = {S[ORC_XX] * gr[0] + S[ORC_XY] * gr[1] + S[ORC_XZ] * gr[2],
                              S[ORC_XY] * gr[0] + S[ORC_YY] * gr[1] + S[ORC_YZ] * gr[2],
                              S[ORC_XZ] * gr[0] + S[ORC_YZ] * gr[1] + S[ORC_ZZ] * gr[2]};
        /* F1, then D2: the corner is one of the 4 corners of the faces on
         * its side of each axis */
        face[0][a] += 0.25 * fl[0] / h;
        face[1][b] += 0.25 * fl[1] / h;
        face[2][c] += 0.25 * fl[2] / h;
      }
  /* F2 N1 */
  double acc = 0.0;
  for (int d = 0; d < 3; ++d) acc += (face[d][1] - face[d][0]) / h;
  return acc;
}

void orc_apply27(const int32_t n[3], double h, const uint8_t* mask, const double* D,
                 const double* v, double* out) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n[0]; ++x)
    for (int y = 0; y < n[1]; ++y)
      for (int z = 0; z < n[2]; ++z)
        out[idx3(n, x, y, z)] = apply27_at(n, h, mask, D, v, x, y, z);
}

/* ------------------------------------------------------------------------ */
/* Mitchell-Schaeffer, one explicit Euler step (eqn:ms1, eqn:ms2)            */
/* ------------------------------------------------------------------------ */
static inline void ms_euler(const orc_problem* P, double v, double w, double jstim,
                            double* vs, double* ws) {
  const double j_in = P->exc * v * v * (1.0 - v) * w / P->tau_in;
  const double j_out = -v / P->tau_out;
  const double dw = (v < P->v_gate) ? (1.0 - w) / P->tau_open : -w / P->tau_close;
  *vs = v + P->dt * (j_in + j_out + jstim);
  *ws = w + P->dt * dw;
}

void orc_ionic(const orc_problem* P, const double* v, const double* w,
               const double* jstim, double* vs, double* ws) {
  const int64_t N = nvox(P->n);
  for (int64_t p = 0; p < N; ++p) {
    if (!P->mask[p]) { vs[p] = v[p]; ws[p] = w[p]; continue; }
    ms_euler(P, v[p], w[p], jstim ? jstim[p] : 0.0, &vs[p], &ws[p]);
  }
}

/* stimulus current at t_n = step*dt: sum of amp over stimuli active at t_n
 * whose region holds the (tissue) voxel.  Region: lo <= p < hi and, when
 * radius > 0, |centre(p) - c|^2 <= radius^2 with the squared distance summed
 * in x, y, z order. */
static void stim_field(const orc_problem* P, int64_t step, double* j) {
  const int64_t N = nvox(P->n);
  memset(j, 0, (size_t)N * sizeof(double));
  const double tn = (double)step * P->dt;
  for (int k = 0; k < P->n_stim; ++k) {
    const orc_stim* s = &P->stim[k];
    if (!(s->t_on <= tn && tn < s->t_off)) continue;
    for (int x = s->lo[0]; x < s->hi[0]; ++x)
      for (int y = s->lo[1]; y < s->hi[1]; ++y)
        for (int z = s->lo[2]; z < s->hi[2]; ++z) {
          if (!inside(P->n, x, y, z)) continue;
          const int64_t p = idx3(P->n, x, y, z);
          if (!P->mask[p]) continue;
          if (s->radius > 0.0) {
            const double dx = (x + 0.5) * P->h - s->center[0];
            const double dy = (y + 0.5) * P->h - s->center[1];
            const double dz = (z + 0.5) * P->h - s->center[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 <= s->radius * s->radius)) continue;
          }
          j[p] += s->amp;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* linear algebra helpers (deterministic: fixed-order sums over x slabs)     */
/* ------------------------------------------------------------------------ */
static double dot(const int32_t n[3], const double* a, const double* b) {
  const int64_t slab = (int64_t)n[1] * n[2];
  double* part = (double*)calloc((size_t)n[0], sizeof(double));
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n[0]; ++x) {
    double s = 0.0;
    for (int64_t i = x * slab; i < (x + 1) * slab; ++i) s += a[i] * b[i];
    part[x] = s;
  }
  double s = 0.0;
  for (int x = 0; x < n[0]; ++x) s += part[x];
  free(part);
  return s;
}

typedef struct {
  const orc_problem* P;
  const uint8_t* mask;  /* domain of the D1 operator */
  const double* D1;
  const uint8_t* mask2; /* domain of the D2 operator (kind 1) */
  const double* D2;     /* second tensor field (kind 1) */
  double alpha;         /* kind 0: the operator is I - alpha A(D1) */
  int kind;             /* 0: I - alpha A(D1);  1: -(A(D1) + A(D2)), each over its own domain */
  double* tmp;
} orc_op;

static void op_apply(const orc_op* o, const double* x, double* y) {
  const orc_problem* P = o->P;
  const int64_t N = nvox(P->n);
  if (o->kind == 0) {
    orc_apply(P->n, P->h, o->mask, o->D1, x, y);
    for (int64_t p = 0; p < N; ++p) y[p] = x[p] - o->alpha * y[p];
  } else {
    orc_apply(P->n, P->h, o->mask, o->D1, x, y);
    orc_apply(P->n, P->h, o->mask2, o->D2, x, o->tmp);
    for (int64_t p = 0; p < N; ++p) y[p] = -(y[p] + o->tmp[p]);
  }
}

/* Jacobi-preconditioned conjugate gradients for the symmetric operator o.
 * Stops when ||r||_2 <= rtol ||b||_2.  Returns the iteration count, or -1
 * when maxit was reached. */
static int pcg(const orc_op* o, const double* dinv, const double* b, double* x,
               double rtol, int maxit) {
  const int32_t* n = o->P->n;
  const int64_t N = nvox(n);
  double* r = (double*)malloc((size_t)N * sizeof(double));
  double* z = (double*)malloc((size_t)N * sizeof(double));
  double* p = (double*)malloc((size_t)N * sizeof(double));
  double* q = (double*)malloc((size_t)N * sizeof(double));
  op_apply(o, x, q);
  for (int64_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
  const double bnorm = sqrt(dot(n, b, b));
  double rnorm = sqrt(dot(n, r, r));
  int it = 0;
  if (bnorm == 0.0) {
    /* zero right-hand side: the solution (in the gauge) is zero */
    memset(x, 0, (size_t)N * sizeof(double));
  } else if (!(rnorm <= rtol * bnorm)) {
    for (int64_t i = 0; i < N; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rz = dot(n, r, z);
    for (it = 1; it <= maxit; ++it) {
      op_apply(o, p, q);
      const double alpha = rz / dot(n, p, q);
      for (int64_t i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
      rnorm = sqrt(dot(n, r, r));
      if (rnorm <= rtol * bnorm) break;
      for (int64_t i = 0; i < N; ++i) z[i] = dinv[i] * r[i];
      const double rz_new = dot(n, r, z);
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int64_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    }
    if (it > maxit) it = -1;
  }
  free(r); free(z); free(p); free(q);
  return it;
}

static void project_mean_zero(const int32_t n[3], const uint8_t* m, double* x) {
  const int64_t N = nvox(n);
  double s = 0.0;
  int64_t cnt = 0;
  for (int64_t p = 0; p < N; ++p) if (m[p]) { s += x[p]; ++cnt; }
  const double mean = cnt ? s / (double)cnt : 0.0;
  for (int64_t p = 0; p < N; ++p) x[p] = m[p] ? x[p] - mean : 0.0;
}

/* The elliptic part of eqn:bidomain1, pure Neumann, with sum phi = 0 over its
 * domain.  phi is the extracellular potential on the heart and, with a bath,
 * the body-tissue potential v_o on the bath (continuous across the heart's
 * boundary).  The equation is the sum of the intracellular and extracellular
 * current balances, so its operator is the sum of two operators, each on
 * its own domain:
 *  - A_i: the intracellular tensor on the heart only.  Faces and blocks
 *    that touch a non-heart voxel are dropped, so no intracellular current
 *    crosses the heart's boundary (last line of eqn:bidomain1);
 *  - A_e: over heart + bath, the extracellular tensor D_e on heart voxels
 *    and sig_bath I on bath voxels (Boundary Conditions: the body tissue
 *    conducts with Sigma_o, the normal extracellular current equals the
 *    body current on the heart's boundary, and none leaves the body).  A
 *    face or block that straddles the two takes the mean of its voxel
 *    tensors, like every other face.  Without a bath it is D_e on the heart.
 * The system is -(A_i + A_e) phi = b with b = A_i v* (zero off the heart).
 * phi holds the warm start on entry.  Returns iterations (-1: maxit). */
int orc_solve_elliptic(const orc_problem* P, const double* b_in, double* phi,
                       double rtol, int maxit) {
  const int64_t N = nvox(P->n);
  double* b = (double*)malloc((size_t)N * sizeof(double));
  double* di = (double*)malloc((size_t)N * sizeof(double));
  double* de = (double*)malloc((size_t)N * sizeof(double));
  double* tmp = (double*)malloc((size_t)N * sizeof(double));
  uint8_t* dom = (uint8_t*)malloc((size_t)N);
  double* Deo = NULL;   /* extracellular + bath tensor field */
  for (int64_t p = 0; p < N; ++p) dom[p] = P->mask[p] || (P->bath && P->bath[p]);
  if (P->bath) {
    Deo = (double*)calloc((size_t)6 * (size_t)N, sizeof(double));
    for (int64_t p = 0; p < N; ++p) {
      if (P->mask[p]) {
        for (int c = 0; c < 6; ++c) Deo[c * N + p] = P->De[c * N + p];
      } else if (P->bath[p]) {
        Deo[ORC_XX * N + p] = P->sig_bath;
        Deo[ORC_YY * N + p] = P->sig_bath;
        Deo[ORC_ZZ * N + p] = P->sig_bath;
      }
    }
  }
  const double* De = Deo ? Deo : P->De;
  memcpy(b, b_in, (size_t)N * sizeof(double));
  project_mean_zero(P->n, dom, b);
  orc_diag(P->n, P->h, P->mask, P->Di, di);
  orc_diag(P->n, P->h, dom, De, de);
  for (int64_t p = 0; p < N; ++p) {
    const double k = -(di[p] + de[p]);
    di[p] = (dom[p] && k > 0.0) ? 1.0 / k : 0.0;
  }
  project_mean_zero(P->n, dom, phi);
  const orc_op o = {P, P->mask, P->Di, dom, De, 0.0, 1, tmp};
  const int it = pcg(&o, di, b, phi, rtol, maxit);
  project_mean_zero(P->n, dom, phi);
  free(b); free(di); free(de); free(tmp); free(dom); free(Deo);
  return it;
}

/* The six limb leads from the extracellular potential at the right-arm,
 * left-arm and left-leg electrodes (Cardiac Simulation chapter, Results,
 * ECG): Einthoven's I = LA - RA, II = LL - RA, III = LL - LA and Goldberger's
 * augmented leads aVR = RA - (LA + LL)/2, aVL = LA - (RA + LL)/2,
 * aVF = LL - (RA + LA)/2.  e holds the voxel coordinates of RA, LA, LL. */
void orc_ecg(const int32_t n[3], const double* phi, const int32_t e[9], double out[6]) {
  const double ra = phi[idx3(n, e[0], e[1], e[2])];
  const double la = phi[idx3(n, e[3], e[4], e[5])];
  const double ll = phi[idx3(n, e[6], e[7], e[8])];
  out[0] = la - ra;
  out[1] = ll - ra;
  out[2] = ll - la;
  out[3] = ra - 0.5 * (la + ll);
  out[4] = la - 0.5 * (ra + ll);
  out[5] = ll - 0.5 * (ra + la);
}

/* ------------------------------------------------------------------------ */
/* time stepping                                                             */
/* ------------------------------------------------------------------------ */
static void record_activation(const orc_problem* P, int64_t step, const double* vold,
                              const double* vnew, double* tact) {
  const int64_t N = nvox(P->n);
  const double tn = (double)step * P->dt;
  for (int64_t p = 0; p < N; ++p) {
    if (!P->mask[p] || !isinf(tact[p])) continue;
    if (vold[p] < P->theta && P->theta <= vnew[p])
      tact[p] = tn + P->dt * (P->theta - vold[p]) / (vnew[p] - vold[p]);
  }
}

/* Advance nsteps operator-split steps.  Returns 0, or 1 when some CG solve
 * hit its iteration limit (the state is still advanced). */
int orc_run(const orc_problem* P, orc_state* S, int32_t nsteps, orc_info* info) {
  const int64_t N = nvox(P->n);
  const double h3 = P->h * P->h * P->h;
  double* j = (double*)malloc((size_t)N * sizeof(double));
  double* vs = (double*)malloc((size_t)N * sizeof(double));
  double* ws = (double*)malloc((size_t)N * sizeof(double));
  double* a = (double*)malloc((size_t)N * sizeof(double));
  double* vn = (double*)malloc((size_t)N * sizeof(double));
  double* dinv = NULL;
  double* tmp = (double*)malloc((size_t)N * sizeof(double));
  int rc = 0;
  orc_info inf;
  memset(&inf, 0, sizeof(inf));
  if (P->model == 0 && P->diff == 1) {
    dinv = (double*)malloc((size_t)N * sizeof(double));
    orc_diag(P->n, P->h, P->mask, P->Di, dinv);
    for (int64_t p = 0; p < N; ++p) dinv[p] = 1.0 / (1.0 - P->dt * dinv[p]);
  }
  double* dA = NULL;   /* diagonal of A, for the Jacobi sweeps */
  if (P->model == 0 && P->diff == 2) {
    dA = (double*)malloc((size_t)N * sizeof(double));
    orc_diag(P->n, P->h, P->mask, P->Di, dA);
  }
  for (int32_t s = 0; s < nsteps; ++s) {
    const int64_t step = S->step;
    /* reaction: one explicit Euler step of the ionic model */
    stim_field(P, step, j);
    double qs = 0.0;
    for (int64_t p = 0; p < N; ++p) qs += j[p];
    inf.q_stim += P->dt * h3 * qs;
    orc_ionic(P, S->v, S->w, j, vs, ws);
    /* diffusion */
    if (P->model == 0 && (P->diff == 0 || P->diff == 3)) {
      if (P->diff == 0) orc_apply(P->n, P->h, P->mask, P->Di, vs, a);
      else orc_apply27(P->n, P->h, P->mask, P->Di, vs, a);
      for (int64_t p = 0; p < N; ++p) vn[p] = vs[p] + P->dt * a[p];
    } else if (P->model == 0 && P->diff == 2) {
      /* implicit Euler by a fixed number of Jacobi sweeps (Linear Solver
       * section, "Implicit Euler", eqn:iejac1): with D the diagonal of A and
       * L + U the rest, u^{k+1} = [I - dt D]^-1 [u^t + dt (L + U) u^k],
       * starting from u^0 = u^t, which under operator splitting is v*. */
      memcpy(vn, vs, (size_t)N * sizeof(double));
      for (int32_t k = 0; k < P->jacobi_sweeps; ++k) {
        orc_apply(P->n, P->h, P->mask, P->Di, vn, a);
        for (int64_t p = 0; p < N; ++p) {
          const double lu = a[p] - dA[p] * vn[p];
          tmp[p] = (vs[p] + P->dt * lu) / (1.0 - P->dt * dA[p]);
        }
        memcpy(vn, tmp, (size_t)N * sizeof(double));
      }
      inf.cg_iters += P->jacobi_sweeps;
      if (P->jacobi_sweeps > inf.cg_max) inf.cg_max = P->jacobi_sweeps;
    } else if (P->model == 0) {
      memcpy(vn, vs, (size_t)N * sizeof(double));
      const orc_op o = {P, P->mask, P->Di, NULL, NULL, P->dt, 0, tmp};
      const int it = pcg(&o, dinv, vs, vn, P->cg_rtol, P->cg_maxit);
      if (it < 0) { rc = 1; inf.cg_fail++; inf.cg_iters += P->cg_maxit; }
      else { inf.cg_iters += it; if (it > inf.cg_max) inf.cg_max = it; }
    } else {
      /* bidomain: elliptic solve for phi_e from v*, then the parabolic update */
      orc_apply(P->n, P->h, P->mask, P->Di, vs, a);
      const int it = orc_solve_elliptic(P, a, S->phi, P->cg_rtol, P->cg_maxit);
      if (it < 0) { rc = 1; inf.cg_fail++; inf.cg_iters += P->cg_maxit; }
      else { inf.cg_iters += it; if (it > inf.cg_max) inf.cg_max = it; }
      for (int64_t p = 0; p < N; ++p) tmp[p] = vs[p] + S->phi[p];
      orc_apply(P->n, P->h, P->mask, P->Di, tmp, a);
      for (int64_t p = 0; p < N; ++p) vn[p] = vs[p] + P->dt * a[p];
    }
    record_activation(P, step, S->v, vn, S->tact);
    for (int64_t p = 0; p < N; ++p) {
      S->v[p] = P->mask[p] ? vn[p] : 0.0;
      S->w[p] = P->mask[p] ? ws[p] : 0.0;
    }
    S->step = step + 1;
  }
  double m = 0.0;
  for (int64_t p = 0; p < N; ++p) if (P->mask[p]) m += S->v[p];
  inf.mass = h3 * m;
  if (info) *info = inf;
  free(j); free(vs); free(ws); free(a); free(vn); free(tmp);
  free(dinv); free(dA);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* discrete adjoint of the explicit monodomain step                          */
/* ------------------------------------------------------------------------ */

/* g_q = -dB(mu, v)/ds_q where B is the symmetric bilinear form of E
 * (E(v) = B(v, v), mu^T A v = -B(mu, v)) and the voxel tensors are
 * s_q * D0_q: each face touching q carries 1/2 D0_q, each block 1/4 D0_q. */
static double dB_ds_at(const int32_t n[3], double h, const uint8_t* mask,
                       const double* D0, const double* mu, const double* v,
                       int x, int y, int z) {
  const int64_t N = nvox(n);
  const int64_t p = idx3(n, x, y, z);
  if (!mask[p]) return 0.0;
  const int c[3] = {x, y, z};
  double acc = 0.0;
  for (int d = 0; d < 3; ++d)
    for (int s = -1; s <= 1; s += 2) {
      int q3[3] = {c[0], c[1], c[2]};
      q3[d] += s;
      if (!inside(n, q3[0], q3[1], q3[2])) continue;
      const int64_t q = idx3(n, q3[0], q3[1], q3[2]);
      if (!mask[q]) continue;
      acc += 0.5 * D0[d * N + p] * (mu[q] - mu[p]) * (v[q] - v[p]) / (h * h);
    }
  for (int d = 0; d < 3; ++d)
    for (int e = d + 1; e < 3; ++e) {
      const int comp = offdiag(d, e);
      for (int ad = 0; ad <= 1; ++ad)
        for (int ae = 0; ae <= 1; ++ae) {
          int b[3] = {c[0], c[1], c[2]};
          b[d] -= ad;
          b[e] -= ae;
          int64_t k[2][2];
          int ok = 1;
          for (int i = 0; i <= 1 && ok; ++i)
            for (int jj = 0; jj <= 1 && ok; ++jj) {
              int q3[3] = {b[0], b[1], b[2]};
              q3[d] += i;
              q3[e] += jj;
              if (!inside(n, q3[0], q3[1], q3[2])) { ok = 0; break; }
              k[i][jj] = idx3(n, q3[0], q3[1], q3[2]);
              if (!mask[k[i][jj]]) ok = 0;
            }
          if (!ok) continue;
          const double gdm = (mu[k[1][0]] + mu[k[1][1]] - mu[k[0][0]] - mu[k[0][1]]) / (2.0 * h);
          const double gem = (mu[k[0][1]] + mu[k[1][1]] - mu[k[0][0]] - mu[k[1][0]]) / (2.0 * h);
          const double gdv = (v[k[1][0]] + v[k[1][1]] - v[k[0][0]] - v[k[0][1]]) / (2.0 * h);
          const double gev = (v[k[0][1]] + v[k[1][1]] - v[k[0][0]] - v[k[1][0]]) / (2.0 * h);
          acc += 0.25 * D0[comp * N + p] * (gdm * gev + gdv * gem);
        }
    }
  return acc;
}

/* bilinear-form gradient, exported for tests: out_q = mu^T (dA/ds_q) v */
void orc_dA_ds(const int32_t n[3], double h, const uint8_t* mask, const double* D0,
               const double* mu, const double* v, double* out) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n[0]; ++x)
    for (int y = 0; y < n[1]; ++y)
      for (int z = 0; z < n[2]; ++z)
        out[idx3(n, x, y, z)] = -dB_ds_at(n, h, mask, D0, mu, v, x, y, z);
}

/* Loss L = sum over voxels activated both in the run and in the target of
 * (T - T*)^2, and its gradient with respect to the per-voxel scale s.
 * P->Di must hold s * D0.  The forward run is explicit monodomain from
 * (v0, w0) at step0 with T_act initialised to +inf; all states are kept.
 * The gate-switch derivative (a Dirac at v = v_gate) is dropped. */
int orc_adjoint(const orc_problem* P, const double* D0, const double* v0,
                const double* w0, int64_t step0, int32_t nsteps,
                const double* tstar, double* grad, double* loss, int64_t* n_used,
                double* tact_out) {
  const int64_t N = nvox(P->n);
  double* V = (double*)malloc((size_t)N * (nsteps + 1) * sizeof(double));
  double* W = (double*)malloc((size_t)N * (nsteps + 1) * sizeof(double));
  double* j = (double*)malloc((size_t)N * sizeof(double));
  double* vs = (double*)malloc((size_t)N * sizeof(double));
  double* ws = (double*)malloc((size_t)N * sizeof(double));
  double* a = (double*)malloc((size_t)N * sizeof(double));
  double* tact = (double*)malloc((size_t)N * sizeof(double));
  int64_t* cross = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  if (!V || !W || !j || !vs || !ws || !a || !tact || !cross) return -1;
  memcpy(V, v0, (size_t)N * sizeof(double));
  memcpy(W, w0, (size_t)N * sizeof(double));
  for (int64_t p = 0; p < N; ++p) { tact[p] = INFINITY; cross[p] = -1; }
  /* forward */
  for (int32_t s = 0; s < nsteps; ++s) {
    const double* v = V + (size_t)s * N;
    const double* w = W + (size_t)s * N;
    double* vn = V + (size_t)(s + 1) * N;
    double* wn = W + (size_t)(s + 1) * N;
    stim_field(P, step0 + s, j);
    orc_ionic(P, v, w, j, vs, ws);
    orc_apply(P->n, P->h, P->mask, P->Di, vs, a);
    for (int64_t p = 0; p < N; ++p) {
      vn[p] = P->mask[p] ? vs[p] + P->dt * a[p] : 0.0;
      wn[p] = P->mask[p] ? ws[p] : 0.0;
    }
    const double tn = (double)(step0 + s) * P->dt;
    for (int64_t p = 0; p < N; ++p) {
      if (!P->mask[p] || cross[p] >= 0) continue;
      if (v[p] < P->theta && P->theta <= vn[p]) {
        tact[p] = tn + P->dt * (P->theta - v[p]) / (vn[p] - v[p]);
        cross[p] = s;
      }
    }
  }
  /* loss */
  double L = 0.0;
  int64_t used = 0;
  for (int64_t p = 0; p < N; ++p)
    if (P->mask[p] && cross[p] >= 0 && isfinite(tstar[p])) {
      L += (tact[p] - tstar[p]) * (tact[p] - tstar[p]);
      ++used;
    }
  /* backward */
  double* av = (double*)calloc((size_t)N, sizeof(double));
  double* aw = (double*)calloc((size_t)N, sizeof(double));
  double* nu = (double*)malloc((size_t)N * sizeof(double));
  double* gs = (double*)malloc((size_t)N * sizeof(double));
  memset(grad, 0, (size_t)N * sizeof(double));
  for (int32_t s = nsteps - 1; s >= 0; --s) {
    const double* v = V + (size_t)s * N;
    const double* w = W + (size_t)s * N;
    const double* vn = V + (size_t)(s + 1) * N;
    /* seed from T's dependence on v_{n+1} for crossings at this step */
    for (int64_t p = 0; p < N; ++p)
      if (cross[p] == s && P->mask[p] && isfinite(tstar[p])) {
        const double dl = 2.0 * (tact[p] - tstar[p]);
        const double del = vn[p] - v[p];
        av[p] += dl * (-P->dt * (P->theta - v[p]) / (del * del));
      }
    /* recompute v* of this step */
    stim_field(P, step0 + s, j);
    orc_ionic(P, v, w, j, vs, ws);
    /* gradient: g_q += dt mu^T (dA/ds_q) v*, mu = dL/dv_{n+1} */
    orc_dA_ds(P->n, P->h, P->mask, D0, av, vs, gs);
    for (int64_t p = 0; p < N; ++p) grad[p] += P->dt * gs[p];
    /* nu = (I + dt A)^T mu = mu + dt A mu */
    orc_apply(P->n, P->h, P->mask, P->Di, av, a);
    for (int64_t p = 0; p < N; ++p) nu[p] = P->mask[p] ? av[p] + P->dt * a[p] : 0.0;
    /* through the ionic step */
    for (int64_t p = 0; p < N; ++p) {
      if (!P->mask[p]) { av[p] = 0.0; aw[p] = 0.0; continue; }
      const double vv = v[p], ww = w[p];
      const double dvs_dv = 1.0 + P->dt * (P->exc * (2.0 * vv - 3.0 * vv * vv) * ww / P->tau_in
                                           - 1.0 / P->tau_out);
      const double dvs_dw = P->dt * P->exc * vv * vv * (1.0 - vv) / P->tau_in;
      const double dws_dw = (vv < P->v_gate) ? 1.0 - P->dt / P->tau_open
                                             : 1.0 - P->dt / P->tau_close;
      const double nav = nu[p] * dvs_dv;
      const double naw = nu[p] * dvs_dw + aw[p] * dws_dw;
      av[p] = nav;
      aw[p] = naw;
    }
    /* seed from T's dependence on v_n for crossings at this step */
    for (int64_t p = 0; p < N; ++p)
      if (cross[p] == s && P->mask[p] && isfinite(tstar[p])) {
        const double dl = 2.0 * (tact[p] - tstar[p]);
        const double del = vn[p] - v[p];
        av[p] += dl * (P->dt * (P->theta - vn[p]) / (del * del));
      }
  }
  *loss = L;
  *n_used = used;
  if (tact_out) memcpy(tact_out, tact, (size_t)N * sizeof(double));
  free(V); free(W); free(j); free(vs); free(ws); free(a); free(tact); free(cross);
  free(av); free(aw); free(nu); free(gs);
  return 0;
}

/* Number of threads the oracle's OpenMP loops run with (the CPU baseline
 * reports it as the cores it used), and a way to change it (the baseline's
 * one-thread figure). */
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n >= 1) omp_set_num_threads(n); }

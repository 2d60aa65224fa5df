// HIP kernels of liblsx for MI355X (gfx950, CDNA4, wave64).
//
// Exact-flow layer splitting on the lifted plane-wave coefficients
// (Wang, Chen, Zhou & Zhou, arXiv 2103.14897, Secs. 3-4, App. A):
//   * fibre Hamiltonian assembly      H_j(fibre) = (1-kappa)/2 D + V^j     (eqs. 3.5-3.6)
//   * batched FP64 Jacobi eigensolver (one workgroup per fibre, any length)
//   * propagator formation            P(t) = U exp(-i t Lambda) U^H
//   * kinetic phase                   c_i <- exp(-i kappa t |K_i|^2/2) c_i  (Alg. 3 step 1)
//   * fibre passes                    X_f <- P_f X_f for all fibres of a layer (Alg. 2 steps 1/2)
//                                     as grouped complex GEMMs on MFMA (FP64, FP32, BF16x3)
//   * FP64 reductions                 mass (eq. 2.3), energy (eq. 2.4), fibre masses
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>

#include "lsx_internal.h"

namespace lsx {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even (finite inputs only)
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// three-term bf16 split of a double: x ~= t0 + t1 + t2
__device__ __forceinline__ void split3(double x, unsigned short& t0, unsigned short& t1, unsigned short& t2) {
  t0 = f2bf((float)x);
  double r = x - (double)bf2f(t0);
  t1 = f2bf((float)r);
  r = r - (double)bf2f(t1);
  t2 = f2bf((float)r);
}
// exact three-term bf16 split of an fp32 value: t0 is x with the low 16 bits cleared, t1 the
// same for the remainder x - t0 (exact in fp32, at most 16 significant bits), and the second
// remainder has at most 8 significant bits, so it is a bf16 itself: t0 + t1 + t2 = x exactly.
// Three masks and two subtractions, against three roundings for split3f.
__device__ __forceinline__ void split3x(float x, unsigned short& t0, unsigned short& t1, unsigned short& t2) {
  const unsigned u = __float_as_uint(x);
  const float r1 = x - __uint_as_float(u & 0xFFFF0000u);
  const unsigned v = __float_as_uint(r1);
  const float r2 = r1 - __uint_as_float(v & 0xFFFF0000u);
  t0 = (unsigned short)(u >> 16);
  t1 = (unsigned short)(v >> 16);
  t2 = (unsigned short)(__float_as_uint(r2) >> 16);
}

// same split from an fp32 value (all residuals exact in fp32)
__device__ __forceinline__ void split3f(float x, unsigned short& t0, unsigned short& t1, unsigned short& t2) {
  t0 = f2bf(x);
  float r = x - bf2f(t0);
  t1 = f2bf(r);
  r = r - bf2f(t1);
  t2 = f2bf(r);
}

template <int BS>
__device__ double block_sum(double v, double* sh) {
  // deterministic tree sum over a block of BS threads
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- assembly (eq. 3.6 on one fibre)
// A (ndim x ndim, row-major) <- H_j restricted to fibre f, or for complex H its real
// embedding [[Re H, -Im H], [Im H, Re H]]; padding rows/cols are zero.  Row i's lifted
// index is mn[i*stride ...]; layer j's own block starts at entry `own`; the kinetic share
// on the diagonal is kfac |K|^2 with kfac = (1 - kappa) / (2 nl) for nl layers.
// Block b assembles fibre fid[b] into its own slot b.
__global__ void k_assemble(const int32_t* fid, const int32_t* ptr, const int32_t* rows, const int32_t* mn, int d,
                           int stride, int own, double kfac, const double* K2, int nv, const int32_t* vidx,
                           const double* vre, const double* vim, int embed, double* Aall, const int64_t* moff,
                           const int32_t* ndim) {
  const int b = blockIdx.x;
  const int f = fid[b];
  const int r0 = ptr[f], L = ptr[f + 1] - r0;
  const int n = ndim[b];
  double* A = Aall + moff[b];
  const int La = embed ? 2 * L : L;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
    const int a = (int)(e / n), b = (int)(e % n);
    double val = 0.0;
    if (a < La && b < La) {
      const int ar = a % L, br = b % L, qa = a / L, qb = b / L;
      const int ia = rows[r0 + ar], ib = rows[r0 + br];
      double hr = 0.0, hi = 0.0;
      for (int v = 0; v < nv; ++v) {
        bool match = true;
        for (int k = 0; k < d; ++k)
          match = match && (mn[(int64_t)ia * stride + own + k] - mn[(int64_t)ib * stride + own + k] == vidx[v * d + k]);
        if (match) {
          hr += vre[v];
          hi += vim[v];
        }
      }
      if (ar == br) hr += kfac * K2[ia];
      if (!embed) val = hr;
      else val = (qa == qb) ? hr : (qa == 0 ? -hi : hi);
    }
    A[e] = val;
  }
}

// ---------------------------------------------------------------- batched cyclic Jacobi
// One workgroup per fibre.  Round-robin (circle) ordering: in round r the pairs are
// (n-1, r) and ((r+i) mod (n-1), (r-i) mod (n-1)), i = 1..n/2-1, all disjoint, so a round
// is A <- J^T A J with J a product of n/2 independent plane rotations.  The update is
// done one 2x2 block at a time (block (i,j) depends only on rotations i and j), which
// needs no barrier between the row and the column transformation.  VT holds V^T, so
// H = V diag(lambda) V^T on exit, eigenvalues in the diagonal of A.
// Last step of both Jacobi solvers.  Each rotation is orthogonal only up to the rounding of
// (c, s): near-degenerate pairs (potential-only fibres) take 45-degree rotations with
// c = s = fl(1/sqrt 2), and 2 fl(1/sqrt 2)^2 = 1 + 2^-52, so both rows grow by the same factor and
// thousands of such rotations per row leave V scaled-orthogonal, V = Q diag(nu), and
// A = diag(nu) Q^T H Q diag(nu).  Normalising each eigenvector (row of V^T) and dividing its
// diagonal entry by nu^2 recovers Q and the eigenvalues.  One workgroup of BS threads.
template <int BS>
__device__ void jacobi_finish(const double* A, double* VT, int n, double* lamf) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  for (int k = wv; k < n; k += BS / 64) {
    double s = 0.0;
    for (int c = lane; c < n; c += 64) {
      const double x = VT[(int64_t)k * n + c];
      s += x * x;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const double r = 1.0 / sqrt(s);
    for (int c = lane; c < n; c += 64) VT[(int64_t)k * n + c] *= r;
    if (lane == 0) lamf[k] = A[(int64_t)k * n + k] / s;
  }
}

// sel (nullable): workgroup i solves matrix sel[i] (else matrix i).
template <int BS>
__global__ __launch_bounds__(BS) void k_jacobi(double* Aall, double* VTall, const int64_t* moff,
                                               const int32_t* ndim, double* lam, const int64_t* loff,
                                               int32_t* info, int maxsweeps, const int32_t* sel) {
  const int f = sel ? sel[blockIdx.x] : blockIdx.x;
  const int n = ndim[f];
  double* A = Aall + moff[f];
  double* VT = VTall + moff[f];
  extern __shared__ double sh[];
  const int np = n / 2;
  double* rc = sh;
  double* rs = sh + np;
  int* rp = reinterpret_cast<int*>(sh + 2 * np);
  int* rq = rp + np;
  __shared__ double red[BS];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;

  for (int64_t e = tid; e < nn; e += BS) VT[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
  double s2 = 0.0;
  for (int64_t e = tid; e < nn; e += BS) s2 += A[e] * A[e];
  const double normF = sqrt(block_sum<BS>(s2, red));
  // rotations are skipped below 1e-16 of the pair's diagonal scale plus 1e-16 ||H||_F:
  // the absolute term sits at rounding-noise level, so matrices with zero diagonal
  // (potential-only fibres) converge instead of rotating noise until the sweep limit
  const double tiny = 1e-16 * normF;

  int sweep = 0;
  bool done = (n < 2);
  for (; sweep < maxsweeps && !done; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    const int m = n - 1;
    for (int r = 0; r < m; ++r) {
      for (int i = tid; i < np; i += BS) {
        const int p = (i == 0) ? m : (r + i) % m;
        const int q = (i == 0) ? r : (r - i + m) % m;
        const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q], apq = A[(int64_t)p * n + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-16 * sqrt(fabs(app * aqq)) + tiny) {
          const double th = (aqq - app) / (2.0 * apq);
          const double t = (fabs(th) > 1e150) ? 0.5 / th
                                              : ((th >= 0.0) ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          rotated = 1;
        }
        rc[i] = c;
        rs[i] = s;
        rp[i] = p;
        rq[i] = q;
      }
      __syncthreads();
      const int nb = np * np;
      for (int idx = tid; idx < nb; idx += BS) {
        const int i = idx / np, j = idx - (idx / np) * np;
        const double ci = rc[i], si = rs[i], cj = rc[j], sj = rs[j];
        if (si == 0.0 && sj == 0.0) continue;
        const int64_t p = rp[i], q = rq[i], p2 = rp[j], q2 = rq[j];
        const double a = A[p * n + p2], b = A[p * n + q2], cc = A[q * n + p2], dd = A[q * n + q2];
        const double a1 = ci * a - si * cc, b1 = ci * b - si * dd;
        const double c1 = si * a + ci * cc, d1 = si * b + ci * dd;
        double a2 = cj * a1 - sj * b1, b2 = sj * a1 + cj * b1;
        double c2 = cj * c1 - sj * d1, d2 = sj * c1 + cj * d1;
        if (i == j) {
          b2 = 0.0;
          c2 = 0.0;
        }
        A[p * n + p2] = a2;
        A[p * n + q2] = b2;
        A[q * n + p2] = c2;
        A[q * n + q2] = d2;
      }
      const int nv = np * n;
      for (int idx = tid; idx < nv; idx += BS) {
        const int i = idx / n, col = idx - (idx / n) * n;
        const double s = rs[i];
        if (s == 0.0) continue;
        const double c = rc[i];
        const int64_t p = rp[i], q = rq[i];
        const double x = VT[p * n + col], y = VT[q * n + col];
        VT[p * n + col] = c * x - s * y;
        VT[q * n + col] = s * x + c * y;
      }
      __syncthreads();
    }
    done = (rotated == 0);
    __syncthreads();
  }
  jacobi_finish<BS>(A, VT, n, lam + loff[f]);
  if (tid == 0) info[f] = done ? sweep : -1;
}

// ---------------------------------------------------------------- blocked two-sided Jacobi
// For long fibres.  A matrix of padded size n (a multiple of 32; padding rows and columns are
// zero and are never rotated) is cut into nb = n/16 blocks of 16 rows.  A round pairs the
// blocks with the same circle method the scalar solver uses for rows, into nb/2 disjoint pairs
// P = (I, J).  For every pair the 32x32 diagonal subproblem A[P, P] takes one cyclic Jacobi
// sweep in LDS, whose rotations accumulate into Q_P; then every 32x32 tile of A and of V^T is
// replaced, A[P, P'] <- Q_P^T A[P, P'] Q_P' and V^T[P, R] <- Q_P^T V^T[P, R] (R: 32 columns).
// Each output tile depends only on its own input tile and two rotations, so a round is two
// launches with no other synchronisation, and the tile products run on the FP64 matrix cores.
// A sweep with no rotation in any subproblem leaves every off-diagonal entry below the same
// threshold as the scalar solver's; the same rotation formula and final normalisation apply.

// slot a of a prefix-sum table with pfx[a] <= item < pfx[a + 1] (pfx[0] = 0, item < pfx[count])
__device__ __forceinline__ int bj_slot(const int32_t* pfx, int count, int item) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pfx[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

// blocks (I, J) of pair i in round r of nb blocks (circle method, nb even)
__device__ __forceinline__ void bj_pair(int nb, int r, int i, int& I, int& J) {
  const int M = nb - 1;
  if (i == 0) {
    I = M;
    J = r;
  } else {
    I = (r + i) % M;
    J = (r - i + M) % M;
  }
}

__global__ __launch_bounds__(1024) void k_bj_init(BJArgs g, const int32_t* sel) {
  const int m = sel[blockIdx.x];
  const int n = g.ndim[m];
  const double* A = g.A + g.moff[m];
  double* VT = g.VT + g.moff[m];
  __shared__ double red[1024];
  const int64_t nn = (int64_t)n * n;
  double s2 = 0.0;
  for (int64_t e = threadIdx.x; e < nn; e += 1024) {
    VT[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
    s2 += A[e] * A[e];
  }
  const double normF = sqrt(block_sum<1024>(s2, red));
  if (threadIdx.x == 0) g.tiny[m] = 1e-16 * normF;
}

__global__ __launch_bounds__(256) void k_bj_pairs(BJArgs g) {
  __shared__ double S[32][33];
  __shared__ double Qs[32][33];
  __shared__ double rc[16], rs[16];
  __shared__ int rp[16], rq[16];
  __shared__ int rot;
  const int item = blockIdx.x;
  const int a = bj_slot(g.pfx_pairs, g.count, item);
  const int m = g.mat[a];
  const int i = item - g.pfx_pairs[a];
  const int n = g.ndim[m];
  int I, J;
  bj_pair(n >> 4, g.round, i, I, J);
  const double* A = g.A + g.moff[m];
  const int tid = threadIdx.x;
  if (tid == 0) rot = 0;
  for (int e = tid; e < 1024; e += 256) {
    const int x = e >> 5, y = e & 31;
    const int gx = (x < 16 ? I : J) * 16 + (x & 15), gy = (y < 16 ? I : J) * 16 + (y & 15);
    S[x][y] = A[(int64_t)gx * n + gy];
    Qs[x][y] = (x == y) ? 1.0 : 0.0;
  }
  const double tiny = g.tiny[m];
  __syncthreads();
  for (int r = 0; r < 31; ++r) {
    if (tid < 16) {
      const int p = (tid == 0) ? 31 : (r + tid) % 31;
      const int q = (tid == 0) ? r : (r - tid + 31) % 31;
      const double app = S[p][p], aqq = S[q][q], apq = S[p][q];
      double c = 1.0, sn = 0.0;
      if (fabs(apq) > 1e-16 * sqrt(fabs(app * aqq)) + tiny) {
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (fabs(th) > 1e150) ? 0.5 / th
                                            : ((th >= 0.0) ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        c = 1.0 / sqrt(t * t + 1.0);
        sn = t * c;
        rot = 1;
      }
      rc[tid] = c;
      rs[tid] = sn;
      rp[tid] = p;
      rq[tid] = q;
    }
    __syncthreads();
    {
      // S <- J^T S J one 2x2 block per thread: rows (p_bi, q_bi), columns (p_bj, q_bj)
      const int bi = tid >> 4, bj = tid & 15;
      const double ci = rc[bi], si = rs[bi], cj = rc[bj], sj = rs[bj];
      if (si != 0.0 || sj != 0.0) {
        const int p = rp[bi], q = rq[bi], p2 = rp[bj], q2 = rq[bj];
        const double a0 = S[p][p2], b0 = S[p][q2], c0 = S[q][p2], d0 = S[q][q2];
        const double a1 = ci * a0 - si * c0, b1 = ci * b0 - si * d0;
        const double c1 = si * a0 + ci * c0, d1 = si * b0 + ci * d0;
        double a2 = cj * a1 - sj * b1, b2 = sj * a1 + cj * b1;
        double c2 = cj * c1 - sj * d1, d2 = sj * c1 + cj * d1;
        if (bi == bj) {
          b2 = 0.0;
          c2 = 0.0;
        }
        S[p][p2] = a2;
        S[p][q2] = b2;
        S[q][p2] = c2;
        S[q][q2] = d2;
      }
      // Q <- Q J: columns (p_k, q_k) of rows x and x + 16
      const int k = tid & 15, x0 = tid >> 4;
      const double c = rc[k], sn = rs[k];
      if (sn != 0.0) {
        const int p = rp[k], q = rq[k];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int x = x0 + 16 * h;
          const double u = Qs[x][p], v = Qs[x][q];
          Qs[x][p] = c * u - sn * v;
          Qs[x][q] = sn * u + c * v;
        }
      }
    }
    __syncthreads();
  }
  double* Qo = g.Q + ((int64_t)g.pfx_pairs[a] + i) * 1024;
  for (int e = tid; e < 1024; e += 256) Qo[e] = Qs[e >> 5][e & 31];
  if (tid == 0 && rot) g.flag[m] = 1;
}

// One wave per 32x32 tile, four tiles per workgroup.  v_mfma_f64_16x16x4f64 takes A as lane l =
// A[l % 16][l / 16] and B as B[l / 16][l % 16] of a 16x4 / 4x16 step and leaves C[4 r + l / 16]
// [l % 16] in element r, so the accumulators of X = A_t Q_P' are, element for element, the B
// operands of the second product Q_P^T X.
__global__ __launch_bounds__(256) void k_bj_tiles(BJArgs g, int total) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + wv;
  if (item >= total) return;
  const int a = bj_slot(g.pfx_tiles, g.count, item);
  const int m = g.mat[a];
  const int t = item - g.pfx_tiles[a];
  const int n = g.ndim[m], nb = n >> 4, np = nb >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const double* Qb = g.Q + (int64_t)g.pfx_pairs[a] * 1024;
  const v4d zero4 = {0.0, 0.0, 0.0, 0.0};
  v4d T[2][2] = {{zero4, zero4}, {zero4, zero4}};
  if (t < np * np) {
    const int P = t / np, P2 = t - (t / np) * np;
    int I, J, I2, J2;
    bj_pair(nb, g.round, P, I, J);
    bj_pair(nb, g.round, P2, I2, J2);
    double* A = g.A + g.moff[m];
    const double* Q1 = Qb + (int64_t)P * 1024;
    const double* Q2 = Qb + (int64_t)P2 * 1024;
    v4d X[2][2] = {{zero4, zero4}, {zero4, zero4}};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 4 * s + lk;
      const int gc = (k < 16 ? I2 : J2) * 16 + (k & 15);
      const double a0 = A[(int64_t)(I * 16 + li) * n + gc];
      const double a1 = A[(int64_t)(J * 16 + li) * n + gc];
      const double b0 = Q2[k * 32 + li], b1 = Q2[k * 32 + 16 + li];
      X[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, X[0][0], 0, 0, 0);
      X[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, X[0][1], 0, 0, 0);
      X[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, X[1][0], 0, 0, 0);
      X[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, X[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 4 * s + lk;
      const double q0 = Q1[k * 32 + li], q1 = Q1[k * 32 + 16 + li];
      const double x0 = X[s >> 2][0][s & 3], x1 = X[s >> 2][1][s & 3];
      T[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(q0, x0, T[0][0], 0, 0, 0);
      T[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(q0, x1, T[0][1], 0, 0, 0);
      T[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(q1, x0, T[1][0], 0, 0, 0);
      T[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(q1, x1, T[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          A[(int64_t)((bi ? J : I) * 16 + 4 * r + lk) * n + (bj ? J2 : I2) * 16 + li] = T[bi][bj][r];
  } else {
    const int tv = t - np * np;
    const int P = tv / np, R = tv - (tv / np) * np;
    int I, J;
    bj_pair(nb, g.round, P, I, J);
    double* VT = g.VT + g.moff[m];
    const double* Q1 = Qb + (int64_t)P * 1024;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 4 * s + lk;
      const int64_t gk = (int64_t)((k < 16 ? I : J) * 16 + (k & 15)) * n + R * 32;
      const double q0 = Q1[k * 32 + li], q1 = Q1[k * 32 + 16 + li];
      const double v0 = VT[gk + li], v1 = VT[gk + 16 + li];
      T[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(q0, v0, T[0][0], 0, 0, 0);
      T[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(q0, v1, T[0][1], 0, 0, 0);
      T[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(q1, v0, T[1][0], 0, 0, 0);
      T[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(q1, v1, T[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          VT[(int64_t)((bi ? J : I) * 16 + 4 * r + lk) * n + R * 32 + 16 * bj + li] = T[bi][bj][r];
  }
}

__global__ __launch_bounds__(1024) void k_bj_finish(BJArgs g, const int32_t* sel, double* lam, const int64_t* loff) {
  const int m = sel[blockIdx.x];
  const int n = g.ndim[m];
  jacobi_finish<1024>(g.A + g.moff[m], g.VT + g.moff[m], n, lam + loff[m]);
}

hipError_t launch_bj_init(hipStream_t s, int nsel, const int32_t* sel, const BJArgs& g) {
  if (nsel == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bj_init, dim3(nsel), dim3(1024), 0, s, g, sel);
  return hipGetLastError();
}

hipError_t launch_bj_round(hipStream_t s, int npairs, int ntiles, const BJArgs& g) {
  if (npairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bj_pairs, dim3(npairs), dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bj_tiles, dim3((ntiles + 3) / 4), dim3(256), 0, s, g, ntiles);
  return hipGetLastError();
}

hipError_t launch_bj_finish(hipStream_t s, int nsel, const int32_t* sel, const BJArgs& g, double* lam,
                            const int64_t* loff) {
  if (nsel == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bj_finish, dim3(nsel), dim3(1024), 0, s, g, sel, lam, loff);
  return hipGetLastError();
}

// f(lambda) = g + i h of one sub-step of length t for each eigenvalue:
//   flow 0 (exact flow)        exp(-i t lambda)
//   flow 1 (backward Euler)    1 / (1 + i t lambda)                     (Alg. 2)
//   flow 2 (Crank-Nicolson)    (1 - i t lambda / 2) / (1 + i t lambda / 2)  (eq. 4.6)
__global__ void k_eig_fn(int64_t nlam, const double* lam, double t, int flow, double2* gh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nlam) {
    const double x = t * lam[i];
    double g, h;
    if (flow == 0) {
      double sn, cn;
      sincos(x, &sn, &cn);
      g = cn;
      h = -sn;
    } else if (flow == 1) {
      const double den = 1.0 + x * x;
      g = 1.0 / den;
      h = -x / den;
    } else {
      const double q = 0.25 * x * x, den = 1.0 + q;
      g = (1.0 - q) / den;
      h = -x / den;
    }
    gh[i] = make_double2(g, h);
  }
}

// ---------------------------------------------------------------- propagator formation
// P(t) = f(H) = sum_k V[.][k] f(lambda_k) V[.][k]^T with f = g + i h.  For an embedded
// complex H (real form M = [[Re H, -Im H], [Im H, Re H]]), g(M) and h(M) hold Re/Im of g(H)
// and h(H) in their left blocks (C_A, C_B and S_A, S_B), so P = (C_A - S_B) + i (C_B + S_A).
// Block b forms fibre fid[b] (slot b); the mixed formats' diagonal goes to positions ptr[f]+a.
template <int FMT>
__global__ void k_form(const int32_t* fid, const int32_t* ptr, const double* VTall, const int64_t* moff,
                       const int32_t* ndim, const int32_t* embed, const double2* ghall, const int64_t* loff,
                       void* Pall, const int64_t* poff, double2* diag) {
  const int b = blockIdx.x;
  const int f = fid[b];
  const int r0 = ptr[f], L = ptr[f + 1] - r0;
  const int n = ndim[b];
  const int emb = embed[b];
  const double* VT = VTall + moff[b];
  const double2* gh = ghall + loff[b];
  char* P = reinterpret_cast<char*>(Pall) + poff[b];
  const int LL = L * L;
  for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < LL; e += gridDim.y * blockDim.x) {
    const int a = e / L, bb = e - (e / L) * L;
    double CA = 0.0, SA = 0.0, CB = 0.0, SB = 0.0;
    for (int k = 0; k < n; ++k) {
      const double2 c = gh[k];
      const double v = VT[(int64_t)k * n + bb];
      const double uv = VT[(int64_t)k * n + a] * v;
      CA += uv * c.x;
      SA += uv * c.y;
      if (emb) {
        const double u2v = VT[(int64_t)k * n + L + a] * v;
        CB += u2v * c.x;
        SB += u2v * c.y;
      }
    }
    const double pr = CA - SB, pi = CB + SA;
    if (FMT == PF_F64) {
      const int Lp = (L + 15) & ~15;
      const int64_t idx = ((int64_t)(a >> 4) * (Lp >> 2) + (bb >> 2)) * 64 + (a & 15) + 16 * (bb & 3);
      reinterpret_cast<double2*>(P)[idx] = make_double2(pr, pi);
    } else if (a == bb) {
      diag[r0 + a] = make_double2(pr, pi);
    } else if (FMT == PF_F32) {
      const int Lp = (L + 15) & ~15;
      const int64_t idx = ((int64_t)(a >> 4) * (Lp >> 2) + (bb >> 2)) * 64 + (a & 15) + 16 * (bb & 3);
      reinterpret_cast<float2*>(P)[idx] = make_float2((float)pr, (float)pi);
    } else {
      const int Lp = (L + 31) & ~31;
      const int64_t chunk = (int64_t)(a >> 4) * (Lp >> 5) + (bb >> 5);
      const int lane = (a & 15) + 16 * ((bb & 31) >> 3), el = bb & 7;
      unsigned short* Q = reinterpret_cast<unsigned short*>(P);
      unsigned short t[6];
      split3(pr, t[0], t[2], t[4]);
      split3(pi, t[1], t[3], t[5]);
#pragma unroll
      for (int pl = 0; pl < 6; ++pl) Q[((chunk * 6 + pl) * 64 + lane) * 8 + el] = t[pl];
    }
  }
}

// ---------------------------------------------------------------- propagator bands
// Over one short step an entry P_ab of a fibre propagator is reached only through chains of
// potential couplings from a to b, each link carrying a factor of order t|v|, so the entries
// fall off quickly away from the diagonal and most column chunks of a row block hold nothing
// a product could feel.  For every 16-row block of every stored propagator this records the
// first and one past the last column chunk (4 columns; 32 for the BF16x3 format) that holds an
// entry with |Re| + |Im| >= tol (for BF16x3 the sum over the three terms' magnitudes bounds
// the entry); a block with no such entry keeps its diagonal chunk.  One workgroup per stored
// propagator; wave w takes row blocks w, w + 4, ...
template <int FMT>
__global__ __launch_bounds__(256) void k_band(const int32_t* fid, const int32_t* ptr, const void* Pall,
                                              const int64_t* poff, const int64_t* boff, double tol,
                                              int32_t* band) {
  constexpr int CW = FMT == PF_BF16X3 ? 32 : 4;
  const int b = blockIdx.x;
  const int f = fid[b];
  const int L = ptr[f + 1] - ptr[f];
  const int Lp = FMT == PF_BF16X3 ? (L + 31) & ~31 : (L + 15) & ~15;
  const int nc = Lp / CW, nrb = (L + 15) >> 4;
  const int lane = threadIdx.x & 63;
  const char* P = reinterpret_cast<const char*>(Pall) + poff[b];
  for (int rb = threadIdx.x >> 6; rb < nrb; rb += blockDim.x >> 6) {
    int lo = -1, hi = -1;
    for (int kc = 0; kc < nc; ++kc) {
      const int64_t ch = (int64_t)rb * nc + kc;
      bool big = false;
      if (FMT == PF_F64) {
        const double2 v = reinterpret_cast<const double2*>(P)[ch * 64 + lane];
        big = fabs(v.x) + fabs(v.y) >= tol;
      } else if (FMT == PF_F32) {
        const float2 v = reinterpret_cast<const float2*>(P)[ch * 64 + lane];
        big = (double)fabsf(v.x) + (double)fabsf(v.y) >= tol;
      } else {
        const v8u16* Q = reinterpret_cast<const v8u16*>(P) + ch * 6 * 64 + lane;
        v8u16 pl[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) pl[k] = Q[k * 64];
#pragma unroll
        for (int el = 0; el < 8; ++el) {
          double m = 0.0;
#pragma unroll
          for (int k = 0; k < 6; ++k) m += fabs((double)bf2f(pl[k][el]));
          big = big || m >= tol;
        }
      }
      if (__any(big)) {
        if (lo < 0) lo = kc;
        hi = kc + 1;
      }
    }
    if (lo < 0) {
      lo = (16 * rb) / CW;
      hi = lo + 1;
    }
    if (lane == 0) {
      band[2 * (boff[b] + rb)] = lo;
      band[2 * (boff[b] + rb) + 1] = hi;
    }
  }
}

// ---------------------------------------------------------------- kinetic phase
__global__ void k_phase_table(int64_t N, const double* K2, double scale, double2* ph) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    double s, c;
    sincos(scale * K2[i], &s, &c);
    ph[i] = make_double2(c, -s);
  }
}

// Thread (r, w) of a workgroup takes column w (and w + TW, ...) of rows r, r + RPB, ... of a
// grid-stride sweep, TW = W rounded up to a power of two (at most 256), RPB = 256 / TW: no
// per-element index division, and every row's phase is loaded once per thread.
__global__ __launch_bounds__(256) void k_phase_apply(int64_t N, int W, int TW, const double2* __restrict__ ph,
                                                     double2* __restrict__ c) {
  const int rpb = 256 / TW;
  const int r = threadIdx.x / TW, w0 = threadIdx.x - r * TW;
  for (int64_t i = (int64_t)blockIdx.x * rpb + r; i < N; i += (int64_t)gridDim.x * rpb) {
    const double2 p = ph[i];
    for (int w = w0; w < W; w += TW) {
      const double2 x = c[i * W + w];
      c[i * W + w] = make_double2(p.x * x.x - p.y * x.y, p.x * x.y + p.y * x.x);
    }
  }
}

// ---------------------------------------------------------------- tile columns
// State column of this lane's slot in each of the tile's NB column blocks (slot
// (wb NB + nb) 16 + lane % 16), and whether it exists.  Column-gathered passes look the
// slot up in the fibre's column list.
template <int NB>
__device__ __forceinline__ void tile_cols(const PassArgs& a, const TileDesc& t, int li, int (&wc)[NB],
                                          bool (&wok)[NB]) {
  const int nc = a.cols ? a.ncols[t.f] : a.W;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int sl = (t.wb * NB + nb) * 16 + li;
    wok[nb] = sl < nc;
    wc[nb] = a.cols ? (wok[nb] ? a.cols[(int64_t)t.f * a.W + sl] : 0) : sl;
  }
}

// ---------------------------------------------------------------- fibre-pass epilogue
// acc[nb][0/1][r]: this lane's part of the 16x16 output blocks, column lane%16 and
// row 4*(lane/16)+r for the FP32-accumulating MFMAs, row 4*r+lane/16 for
// v_mfma_f64_16x16x4f64 (ROWS_F64).  Summed over the KS waves in fixed order; mixed
// formats add the FP64 diagonal term d_a x_a; an optional kinetic phase multiplies
// the output row (the phase sub-step that follows this pass, fused).
// With a.nt set the output is stored non-temporally.  The next pass reads it in the other
// layer's fibre order, mostly on other XCDs, so keeping it in this XCD's L2 can only add
// write-back work at the end of the launch; but for states that fit the last-level cache,
// ordinary stores leave it there for the next pass.  The host measures which is faster.
template <int NB, int KS, bool MIX, bool ROWS_F64>
__device__ __forceinline__ void pass_epilogue(const PassArgs& a, const TileDesc& t, double (&acc)[NB][2][4],
                                              double* red, const int (&wc)[NB], const bool (&wok)[NB]) {
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lk = lane >> 4;
  const int r0 = t.r0, L = t.L, rb = t.rb;
  const int W = a.W;
  if (KS > 1) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(((kw * NB + nb) * 2 + c) * 4 + r) * 64 + lane] = acc[nb][c][r];
    __syncthreads();
  }
  for (int r = (KS > 1 ? kw : 0); r < 4; r += KS) {
    const int arow = 16 * rb + (ROWS_F64 ? 4 * r + lk : 4 * lk + r);
    if (arow >= L) continue;
    const int p = r0 + arow;
    const int64_t orow = a.out_pos ? a.out_pos[p] : p;
    const int64_t irow = a.in_pos ? a.in_pos[p] : p;
    double2 ph = make_double2(1.0, 0.0);
    if (a.ph) ph = a.ph[a.ph_idx ? a.ph_idx[p] : p];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int w = wc[nb];
      if (!wok[nb]) continue;
      double yr, yi;
      if (KS > 1) {
        yr = 0.0;
        yi = 0.0;
        for (int j = 0; j < KS; ++j) {
          yr += red[(((j * NB + nb) * 2 + 0) * 4 + r) * 64 + lane];
          yi += red[(((j * NB + nb) * 2 + 1) * 4 + r) * 64 + lane];
        }
      } else {
        yr = acc[nb][0][r];
        yi = acc[nb][1][r];
      }
      if (MIX || a.wt) {
        const double2 x = a.X[irow * W + w];
        if (MIX) {
          const double2 dg = a.diag[t.d0 + arow];
          yr += dg.x * x.x - dg.y * x.y;
          yi += dg.x * x.y + dg.y * x.x;
        }
        if (a.wt) {
          const double g = a.wt[(int64_t)t.f * W + w];
          yr = x.x + g * (yr - x.x);
          yi = x.y + g * (yi - x.y);
        }
      }
      if (a.ph) {
        const double zr = ph.x * yr - ph.y * yi;
        yi = ph.x * yi + ph.y * yr;
        yr = zr;
      }
      double2* y = a.Y + orow * W + w;
      if (a.nt) {
        // empty compiler barriers (no instruction) around the stores keep them from being
        // hoisted or sunk together with the other branch's, which would drop the hint
        asm volatile("" ::: "memory");
        __builtin_nontemporal_store(yr, &y->x);
        __builtin_nontemporal_store(yi, &y->y);
        asm volatile("" ::: "memory");
      } else {
        *y = make_double2(yr, yi);
      }
    }
  }
}

// ---------------------------------------------------------------- MFMA fibre passes
// Tile = (fibre, 16 output rows rb, 16*NB columns wb).  The KS waves of a workgroup
// take interleaved groups of U k-steps; all loads of a group (propagator chunk and
// state operands) are issued before its MFMAs, so a group pays the memory latency
// once.  When the input array is laid out fibre-contiguously (in_pos null) the state
// operands need no index load at all.

__device__ __forceinline__ int64_t in_row(const PassArgs& a, int p) { return a.in_pos ? a.in_pos[p] : p; }

// Band of a tile in units of `unit` fibre positions (4 for a k-step of the FP64 / FP32
// products, 32 for a BF16x3 chunk): [lo, hi), clamped to the padded fibre length Lp.
__device__ __forceinline__ void tile_band(const TileDesc& t, int Lp, int unit, int& lo, int& hi) {
  lo = t.k0 / unit;
  hi = (min(t.k1, Lp) + unit - 1) / unit;
}

// Operand loads of one group of U k-steps (4 fibre positions each) for the FP64/FP32
// kernels: propagator chunk per k-step (A operand) and NB state values (B operand).
template <typename PT, int NB, int U>
struct Group4 {
  PT p[U];
  double2 x[U][NB];
};

// All operand loads are unconditional: an out-of-range operand (k-step past the tile's
// band end kend, column past W) is read from a zeroed buffer instead, so the address is
// selected, not the value, and no loaded value is consumed before the MFMAs that need
// it -- the loads of the next group stay in flight during the current group.
// GATHER: element k of the fibre is row in_pos[r0 + k] of X, else row r0 + k.
template <bool GATHER>
__device__ __forceinline__ int64_t xrow(const PassArgs& a, int p) {
  return GATHER ? (int64_t)a.in_pos[p] : (int64_t)p;
}

template <bool GATHER, typename PT, int NB, int U>
__device__ __forceinline__ void load_group4(Group4<PT, NB, U>& G, const PassArgs& a, const PT* P, int g, int kend,
                                            int r0, int L, int lk, const int (&wc)[NB], const bool (&wok)[NB]) {
  const PT* zp = reinterpret_cast<const PT*>(a.zero);
  const double2* zx = reinterpret_cast<const double2*>(a.zero);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int ks = g + u, k = 4 * ks + lk;
    G.p[u] = *((ks < kend) ? P + (int64_t)ks * 64 : zp);
    const bool ok = ks < kend && k < L;
    const int64_t row = xrow<GATHER>(a, r0 + (ok ? k : 0));
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) G.x[u][nb] = *((ok && wok[nb]) ? a.X + row * a.W + wc[nb] : zx);
  }
}

// Complex products with three real MFMAs (the 3M / Gauss form): for P = a + ib and
// x = c + id,  k1 = (a + b) c,  k2 = a (d - c),  k3 = b (c + d);  Re = k1 - k3, Im = k1 + k2.
// The sums a + b, d - c, c + d are formed on the VALU in the operand precision.
template <int NB, int U>
__device__ __forceinline__ void mma_group_f64(v4d (&k1)[NB], v4d (&k2)[NB], v4d (&k3)[NB],
                                              const Group4<double2, NB, U>& G) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double ps = G.p[u].x + G.p[u].y;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const double xr = G.x[u][nb].x, xi = G.x[u][nb].y;
      k1[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ps, xr, k1[nb], 0, 0, 0);
      k2[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(G.p[u].x, xi - xr, k2[nb], 0, 0, 0);
      k3[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(G.p[u].y, xr + xi, k3[nb], 0, 0, 0);
    }
  }
}

template <int NB, int U>
__device__ __forceinline__ void mma_group_f32(v4f (&k1)[NB], v4f (&k2)[NB], v4f (&k3)[NB],
                                              const Group4<float2, NB, U>& G) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const float ps = G.p[u].x + G.p[u].y;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float xr = (float)G.x[u][nb].x, xi = (float)G.x[u][nb].y;
      k1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ps, xr, k1[nb], 0, 0, 0);
      k2[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G.p[u].x, xi - xr, k2[nb], 0, 0, 0);
      k3[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G.p[u].y, xr + xi, k3[nb], 0, 0, 0);
    }
  }
}

// ---------------------------------------------------------------- persistent batched launches
// The grid holds what the chip keeps resident (a multiple of 8 workgroups).  The tile list is
// XCD interleaved (tile i belongs to XCD i mod 8) and workgroup b runs on XCD b mod 8.
//  persist = 1: workgroup b takes the tiles i = 8 k + (b mod 8), k = 0, 1, ..., of its XCD's
//    queue through a device atomic counter, so uneven tiles balance dynamically within each
//    XCD; the claim of the next tile is issued before the current tile runs, so its latency
//    overlaps the tile's loads.  queue[0..7] are the per-XCD counters and queue[8] counts
//    finished workgroups; the last workgroup to finish clears all nine, so every launch starts
//    from zeros without a memset node (graph replays).
//  persist = 2: workgroup b takes the tiles b, b + G, b + 2G, ... (G = grid size), no atomics.
// No workgroup waits on another.
template <typename Tile>
__device__ __forceinline__ void persistent_tiles(const PassArgs& a0, Tile&& tile) {
  if (a0.persist == 2) {
    for (int ti = blockIdx.x; ti < a0.ntiles; ti += gridDim.x) {
      tile(ti);
      __syncthreads();  // the tile's LDS is free again
    }
    return;
  }
  __shared__ int next;
  const int x = blockIdx.x & 7;
  if (threadIdx.x == 0) next = 8 * atomicAdd(a0.queue + x, 1) + x;
  __syncthreads();
  int ti = next;
  while (ti < a0.ntiles) {
    int ahead = 0;
    if (threadIdx.x == 0) ahead = 8 * atomicAdd(a0.queue + x, 1) + x;
    tile(ti);
    __syncthreads();  // the tile's LDS and `next` are free again
    if (threadIdx.x == 0) next = ahead;
    __syncthreads();
    ti = next;
  }
  if (threadIdx.x == 0 && atomicAdd(a0.queue + 8, 1) == (int)gridDim.x - 1)
    for (int i = 0; i < 9; ++i) atomicExch(a0.queue + i, 0);
}

// FP64: complex128 P, X on v_mfma_f64_16x16x4f64.  Three independent accumulator chains
// per column block (the 3M products above); groups of U k-steps are double buffered in
// registers, so the loads of group g+1 are in flight during the MFMAs of g.
template <int NB, int KS, int U, bool GATHER, bool BATCH>
__device__ __forceinline__ void k_pass_f64_tile(const PassArgs& a0, int ti, double* red) {
  const TileDesc t = a0.tiles[ti];
  if (t.f < 0) return;
  // batched launches: this tile's system arguments (uniform scalar loads)
  const PassArgs a = BATCH ? a0.batch[t.f] : a0;
  const int r0 = t.r0, L = t.L;
  const int nks = ((L + 15) & ~15) >> 2;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const double2* P = reinterpret_cast<const double2*>(reinterpret_cast<const char*>(a.P) + t.poff) +
                     (int64_t)t.rb * nks * 64 + lane;
  int wc[NB];
  bool wok[NB];
  tile_cols<NB>(a, t, li, wc, wok);
  v4d k1[NB], k2[NB], k3[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) k1[nb] = k2[nb] = k3[nb] = (v4d){0.0, 0.0, 0.0, 0.0};
  // two register buffers in ping-pong: B is loaded while A is consumed and vice versa
  Group4<double2, NB, U> A, B;
  const int stride = KS * U;
  int klo, khi;
  tile_band(t, 4 * nks, 4, klo, khi);
  int g = klo + kw * U;
  load_group4<GATHER>(A, a, P, g, khi, r0, L, lk, wc, wok);
  for (; g < khi; g += 2 * stride) {
    load_group4<GATHER>(B, a, P, g + stride, khi, r0, L, lk, wc, wok);  // past the band: zeros
    __builtin_amdgcn_sched_barrier(0);
    mma_group_f64(k1, k2, k3, A);
    if (g + stride >= khi) break;
    load_group4<GATHER>(A, a, P, g + 2 * stride, khi, r0, L, lk, wc, wok);
    __builtin_amdgcn_sched_barrier(0);
    mma_group_f64(k1, k2, k3, B);
  }
  double acc[NB][2][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[nb][0][r] = k1[nb][r] - k3[nb][r];
      acc[nb][1][r] = k1[nb][r] + k2[nb][r];
    }
  pass_epilogue<NB, KS, false, true>(a, t, acc, red, wc, wok);
}

template <int NB, int KS, int U, bool GATHER, bool BATCH>
__global__ __launch_bounds__(64 * KS) void k_pass_f64(PassArgs a0) {
  extern __shared__ double red[];
  if (a0.tcount && (int)blockIdx.x >= *a0.tcount) return;
  k_pass_f64_tile<NB, KS, U, GATHER, BATCH>(a0, blockIdx.x, red);
}

template <int NB, int KS, int U, bool GATHER>
__global__ __launch_bounds__(64 * KS) void k_pass_f64_persist(PassArgs a0) {
  extern __shared__ double red[];
  persistent_tiles(a0, [&](int ti) { k_pass_f64_tile<NB, KS, U, GATHER, true>(a0, ti, red); });
}

// Mixed FP32: y = d .* x (FP64) + E x~ with E complex64, x~ = fp32(x), FP32 MFMA
// accumulation (v_mfma_f32_16x16x4f32, 3M products), same pipelining as the FP64 kernel.
template <int NB, int KS, int U, bool GATHER, bool BATCH>
__device__ __forceinline__ void k_pass_f32_tile(const PassArgs& a0, int ti, double* red) {
  const TileDesc t = a0.tiles[ti];
  if (t.f < 0) return;
  // batched launches: this tile's system arguments (uniform scalar loads)
  const PassArgs a = BATCH ? a0.batch[t.f] : a0;
  const int r0 = t.r0, L = t.L;
  const int nks = ((L + 15) & ~15) >> 2;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const float2* P = reinterpret_cast<const float2*>(reinterpret_cast<const char*>(a.P) + t.poff) +
                    (int64_t)t.rb * nks * 64 + lane;
  int wc[NB];
  bool wok[NB];
  tile_cols<NB>(a, t, li, wc, wok);
  v4f k1[NB], k2[NB], k3[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) k1[nb] = k2[nb] = k3[nb] = (v4f){0.f, 0.f, 0.f, 0.f};
  Group4<float2, NB, U> A, B;
  const int stride = KS * U;
  int klo, khi;
  tile_band(t, 4 * nks, 4, klo, khi);
  int g = klo + kw * U;
  load_group4<GATHER>(A, a, P, g, khi, r0, L, lk, wc, wok);
  for (; g < khi; g += 2 * stride) {
    load_group4<GATHER>(B, a, P, g + stride, khi, r0, L, lk, wc, wok);  // past the band: zeros
    __builtin_amdgcn_sched_barrier(0);
    mma_group_f32(k1, k2, k3, A);
    if (g + stride >= khi) break;
    load_group4<GATHER>(A, a, P, g + 2 * stride, khi, r0, L, lk, wc, wok);
    __builtin_amdgcn_sched_barrier(0);
    mma_group_f32(k1, k2, k3, B);
  }
  double acc[NB][2][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[nb][0][r] = (double)k1[nb][r] - (double)k3[nb][r];
      acc[nb][1][r] = (double)k1[nb][r] + (double)k2[nb][r];
    }
  pass_epilogue<NB, KS, true, false>(a, t, acc, red, wc, wok);
}

template <int NB, int KS, int U, bool GATHER, bool BATCH>
__global__ __launch_bounds__(64 * KS) void k_pass_f32(PassArgs a0) {
  extern __shared__ double red[];
  if (a0.tcount && (int)blockIdx.x >= *a0.tcount) return;
  k_pass_f32_tile<NB, KS, U, GATHER, BATCH>(a0, blockIdx.x, red);
}

template <int NB, int KS, int U, bool GATHER>
__global__ __launch_bounds__(64 * KS) void k_pass_f32_persist(PassArgs a0) {
  extern __shared__ double red[];
  persistent_tiles(a0, [&](int ti) { k_pass_f32_tile<NB, KS, U, GATHER, true>(a0, ti, red); });
}

// ---------------------------------------------------------------- row-split passes, LDS-staged state
// Workgroup = MS waves on MS consecutive 16-row blocks of one fibre (tile rb counts groups
// of MS blocks) and the same 16 NB columns.  The state operand of every 16-row chunk of
// the fibre is read from memory once per workgroup, converted once (FP32 and the 3M sums
// x_r, x_i - x_r, x_r + x_i) into double-buffered LDS and read there by all MS waves, so
// each state row is fetched once per row-block group instead of once per row block.  Each
// wave streams its own propagator rows, one chunk ahead in registers.  No cross-wave
// reduction: every wave owns its output rows.  Needs MS <= 4 NB.  Chunks are KC k-steps
// (4 KC fibre positions); four- and eight-wave groups take 32-row chunks, which halves the
// barriers and doubles the work that hides each chunk's loads without costing occupancy.
// With band-limited products the staged chunks cover the union of the group's bands, and
// each wave multiplies only the chunks of its own row block's band (PassArgs::rb_band), so
// larger groups read the state operand fewer times without adding products.
template <int NB, int MS>
struct StageMap {
  static constexpr int KC = MS >= 4 ? 8 : 4;   // k-steps per chunk
  static constexpr int CR = 4 * KC;            // rows of a chunk
  static constexpr int CW = 16 * NB;           // columns of a chunk
  static constexpr int PER = CR * CW / (64 * MS);  // elements per thread per chunk
  static constexpr int RSTEP = 64 * MS / CW;   // chunk rows between a thread's elements
};

template <int PER, int RSTEP, int CR, bool GATHER>
__device__ __forceinline__ void stage_load_f32(double2 (&v)[PER], const PassArgs& a, int ch, int r0, int L, int w,
                                               bool wok, int rr0) {
  const double2* zx = reinterpret_cast<const double2*>(a.zero);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int k = CR * ch + rr0 + j * RSTEP;
    const bool ok = wok && k < L;
    const int64_t row = xrow<GATHER>(a, r0 + (ok ? k : 0));
    v[j] = *(ok ? a.X + row * a.W + w : zx);
  }
}

template <int NB, int MS, bool GATHER>
__global__ __launch_bounds__(64 * MS) void k_pass_f32m(PassArgs a) {
  using SM = StageMap<NB, MS>;
  constexpr int KC = SM::KC;
  __shared__ float4 xs[2][SM::CR][SM::CW];
  if (a.tcount && (int)blockIdx.x >= *a.tcount) return;
  const TileDesc t0 = a.tiles[blockIdx.x];
  if (t0.f < 0) return;
  const int r0 = t0.r0, L = t0.L;
  const int nks = ((L + 15) & ~15) >> 2;
  // chunks [clo, clo + nch) cover the tile's band; k-steps past nks read zeros
  int clo, nch;
  tile_band(t0, 4 * nks, SM::CR, clo, nch);
  nch -= clo;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  TileDesc t = t0;
  t.rb = t0.rb * MS + kw;
  const bool act = t.rb < ((L + 15) >> 4);
  const float2* zp = reinterpret_cast<const float2*>(a.zero);
  const float2* P = reinterpret_cast<const float2*>(reinterpret_cast<const char*>(a.P) + t.poff) +
                    (int64_t)(act ? t.rb : 0) * nks * 64 + lane;
  int wc[NB];
  bool wok[NB];
  tile_cols<NB>(a, t, li, wc, wok);
  // this thread's staging slot: column c (fixed), rows rr0 + j RSTEP of each chunk
  const int c = threadIdx.x % SM::CW, rr0 = threadIdx.x / SM::CW;
  int sw;
  bool sok;
  {
    const int nc = a.cols ? a.ncols[t.f] : a.W;
    const int sl = t.wb * SM::CW + c;
    sok = sl < nc;
    sw = a.cols ? (sok ? a.cols[(int64_t)t.f * a.W + sl] : 0) : sl;
  }
  v4f k1[NB], k2[NB], k3[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) k1[nb] = k2[nb] = k3[nb] = (v4f){0.f, 0.f, 0.f, 0.f};
  double2 sv[SM::PER];
  float2 Ac[KC], An[KC];
  // chunks of the band in the order c0, c0 + 1, ... (cyclically), with the workgroup's own
  // rows last: the epilogue's FP64 reload of those rows then finds them in this XCD's L2,
  // just staged
  const int c0 = (((t0.rb + 1) * MS * 16 / SM::CR - clo) % nch + nch) % nch;
  auto chunk = [&](int i) { return clo + (i + c0 < nch ? i + c0 : i + c0 - nch); };
  // this wave's own band [wlo, whi) of chunks (its row block's), inside the staged ones
  int wlo = clo, whi = clo + nch;
  if (a.rb_band && t0.bb >= 0 && act) {
    const int2 wb = reinterpret_cast<const int2*>(a.rb_band)[t0.bb + t.rb];
    wlo = wb.x / SM::CR;
    whi = (min(wb.y, 4 * nks) + SM::CR - 1) / SM::CR;
  }
  auto mine = [&](int cc) { return act && cc >= wlo && cc < whi; };
  stage_load_f32<SM::PER, SM::RSTEP, SM::CR, GATHER>(sv, a, chunk(0), r0, L, sw, sok, rr0);
  {
    const bool in = mine(chunk(0));
#pragma unroll
    for (int u = 0; u < KC; ++u) {
      const int ks = KC * chunk(0) + u;
      Ac[u] = (in && ks < nks) ? P[(int64_t)ks * 64] : *zp;
    }
  }
#pragma unroll
  for (int j = 0; j < SM::PER; ++j) {
    const float xr = (float)sv[j].x, xi = (float)sv[j].y;
    xs[0][rr0 + j * SM::RSTEP][c] = make_float4(xr, xi - xr, xr + xi, 0.f);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) {
      stage_load_f32<SM::PER, SM::RSTEP, SM::CR, GATHER>(sv, a, chunk(ch + 1), r0, L, sw, sok, rr0);
      const bool in = mine(chunk(ch + 1));
#pragma unroll
      for (int u = 0; u < KC; ++u) {
        const int ks = KC * chunk(ch + 1) + u;
        An[u] = (in && ks < nks) ? P[(int64_t)ks * 64] : *zp;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (mine(chunk(ch))) {
#pragma unroll
      for (int u = 0; u < KC; ++u) {
        const float ps = Ac[u].x + Ac[u].y;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float4 b = xs[buf][4 * u + lk][nb * 16 + li];
          k1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ps, b.x, k1[nb], 0, 0, 0);
          k2[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ac[u].x, b.y, k2[nb], 0, 0, 0);
          k3[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ac[u].y, b.z, k3[nb], 0, 0, 0);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < SM::PER; ++j) {
        const float xr = (float)sv[j].x, xi = (float)sv[j].y;
        xs[buf ^ 1][rr0 + j * SM::RSTEP][c] = make_float4(xr, xi - xr, xr + xi, 0.f);
      }
#pragma unroll
      for (int u = 0; u < KC; ++u) Ac[u] = An[u];
    }
    __syncthreads();
  }
  if (!act) return;
  double acc[NB][2][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[nb][0][r] = (double)k1[nb][r] - (double)k3[nb][r];
      acc[nb][1][r] = (double)k1[nb][r] + (double)k2[nb][r];
    }
  pass_epilogue<NB, 1, true, false>(a, t, acc, nullptr, wc, wok);
}

// Mixed BF16x3: E = E0+E1+E2 and x~ = x0+x1+x2 (bf16 terms); the six products E0x0,
// E0x1, E1x0, E0x2, E1x1, E2x0 on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, plus
// the FP64 diagonal term.  A k-step here is a chunk of 32 fibre positions.  Four
// accumulator chains (Er Xr, Ei Xi, Er Xi, Ei Xr); chunk loads are double buffered.
__device__ __forceinline__ v8bf as_bf(const v8u16& u) { return __builtin_bit_cast(v8bf, u); }

template <int NB>
struct ChunkBF {
  v8u16 e[6];
  double2 x[NB][8];
};

template <bool GATHER, int NB>
__device__ __forceinline__ void load_chunk_bf(ChunkBF<NB>& C, const PassArgs& a, const v8u16* P, int kc, int kend,
                                              int r0, int L, int lk, const int (&wc)[NB], const bool (&wok)[NB]) {
  const bool kin = kc < kend;
  const v8u16* zp = reinterpret_cast<const v8u16*>(a.zero);
  const double2* zx = reinterpret_cast<const double2*>(a.zero);
#pragma unroll
  for (int pl = 0; pl < 6; ++pl) C.e[pl] = *(kin ? P + ((int64_t)kc * 6 + pl) * 64 : zp);
#pragma unroll
  for (int el = 0; el < 8; ++el) {
    const int k = 32 * kc + 8 * lk + el;
    const bool ok = kin && k < L;
    const int64_t row = xrow<GATHER>(a, r0 + (ok ? k : 0));
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) C.x[nb][el] = *((ok && wok[nb]) ? a.X + row * a.W + wc[nb] : zx);
  }
}

// acc += A (3 bf16 terms) * B (3 bf16 terms), six cross products, smallest first
__device__ __forceinline__ v4f mma3(v4f c, const v8bf& a0, const v8bf& a1, const v8bf& a2, const v8bf& b0,
                                    const v8bf& b1, const v8bf& b2) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, c, 0, 0, 0);
  return c;
}

template <int NB>
__device__ __forceinline__ void mma_chunk_bf(v4f (&rr)[NB], v4f (&ii)[NB], v4f (&ri)[NB], v4f (&ir)[NB],
                                             const ChunkBF<NB>& C) {
  const v8bf er0 = as_bf(C.e[0]), ei0 = as_bf(C.e[1]), er1 = as_bf(C.e[2]);
  const v8bf ei1 = as_bf(C.e[3]), er2 = as_bf(C.e[4]), ei2 = as_bf(C.e[5]);
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    v8u16 xr0, xr1, xr2, xi0, xi1, xi2;
#pragma unroll
    for (int el = 0; el < 8; ++el) {
      unsigned short a0, a1, a2, b0, b1, b2;
      split3f((float)C.x[nb][el].x, a0, a1, a2);
      split3f((float)C.x[nb][el].y, b0, b1, b2);
      xr0[el] = a0; xr1[el] = a1; xr2[el] = a2;
      xi0[el] = b0; xi1[el] = b1; xi2[el] = b2;
    }
    const v8bf Xr0 = as_bf(xr0), Xr1 = as_bf(xr1), Xr2 = as_bf(xr2);
    const v8bf Xi0 = as_bf(xi0), Xi1 = as_bf(xi1), Xi2 = as_bf(xi2);
    rr[nb] = mma3(rr[nb], er0, er1, er2, Xr0, Xr1, Xr2);
    ii[nb] = mma3(ii[nb], ei0, ei1, ei2, Xi0, Xi1, Xi2);
    ri[nb] = mma3(ri[nb], er0, er1, er2, Xi0, Xi1, Xi2);
    ir[nb] = mma3(ir[nb], ei0, ei1, ei2, Xr0, Xr1, Xr2);
  }
}

template <int NB, int KS, int U, bool GATHER, bool BATCH>
__device__ __forceinline__ void k_pass_bf16x3_tile(const PassArgs& a0, int ti, double* red) {
  const TileDesc t = a0.tiles[ti];
  if (t.f < 0) return;
  // batched launches: this tile's system arguments (uniform scalar loads)
  const PassArgs a = BATCH ? a0.batch[t.f] : a0;
  const int r0 = t.r0, L = t.L;
  const int nkc = ((L + 31) & ~31) >> 5;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const v8u16* P = reinterpret_cast<const v8u16*>(reinterpret_cast<const char*>(a.P) + t.poff) +
                   (int64_t)t.rb * nkc * 6 * 64 + lane;
  int wc[NB];
  bool wok[NB];
  tile_cols<NB>(a, t, li, wc, wok);
  v4f rr[NB], ii[NB], ri[NB], ir[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) rr[nb] = ii[nb] = ri[nb] = ir[nb] = (v4f){0.f, 0.f, 0.f, 0.f};
  ChunkBF<NB> A, B;
  int klo, khi;
  tile_band(t, 32 * nkc, 32, klo, khi);
  int kc = klo + kw;
  load_chunk_bf<GATHER>(A, a, P, kc, khi, r0, L, lk, wc, wok);
  for (; kc < khi; kc += 2 * KS) {
    load_chunk_bf<GATHER>(B, a, P, kc + KS, khi, r0, L, lk, wc, wok);  // past the band: zeros
    __builtin_amdgcn_sched_barrier(0);
    mma_chunk_bf(rr, ii, ri, ir, A);
    if (kc + KS >= khi) break;
    load_chunk_bf<GATHER>(A, a, P, kc + 2 * KS, khi, r0, L, lk, wc, wok);
    __builtin_amdgcn_sched_barrier(0);
    mma_chunk_bf(rr, ii, ri, ir, B);
  }
  double acc[NB][2][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[nb][0][r] = (double)rr[nb][r] - (double)ii[nb][r];
      acc[nb][1][r] = (double)ri[nb][r] + (double)ir[nb][r];
    }
  pass_epilogue<NB, KS, true, false>(a, t, acc, red, wc, wok);
}

template <int NB, int KS, int U, bool GATHER, bool BATCH>
__global__ __launch_bounds__(64 * KS) void k_pass_bf16x3(PassArgs a0) {
  extern __shared__ double red[];
  if (a0.tcount && (int)blockIdx.x >= *a0.tcount) return;
  k_pass_bf16x3_tile<NB, KS, U, GATHER, BATCH>(a0, blockIdx.x, red);
}

template <int NB, int KS, int U, bool GATHER>
__global__ __launch_bounds__(64 * KS) void k_pass_bf16x3_persist(PassArgs a0) {
  extern __shared__ double red[];
  persistent_tiles(a0, [&](int ti) { k_pass_bf16x3_tile<NB, KS, U, GATHER, true>(a0, ti, red); });
}

// Row-split BF16x3 pass: as k_pass_f32m, with 32-row chunks.  The staging threads split each
// state value once (x~ = fp32(x) into three bf16 terms, real and imaginary parts) into six
// LDS planes stored column-major (a lane's 8 consecutive k values are one 16-byte read);
// every wave multiplies its own propagator rows (six bf16 planes, one chunk ahead in
// registers) with the shared planes.  Needs MS <= 8 NB.
template <int NB>
struct StageBF {
  static constexpr int CW = 16 * NB;
  static constexpr int KP = 40;  // padded k stride of a column (32 used)
};

template <int NB, int MS, bool GATHER>
__global__ __launch_bounds__(64 * MS) void k_pass_bf16m(PassArgs a) {
  constexpr int CW = StageBF<NB>::CW, KP = StageBF<NB>::KP;
  constexpr int PER = 32 * CW / (64 * MS), RSTEP = 64 * MS / CW;
  __shared__ __attribute__((aligned(16))) unsigned short xb[2][6][CW][KP];
  if (a.tcount && (int)blockIdx.x >= *a.tcount) return;
  const TileDesc t0 = a.tiles[blockIdx.x];
  if (t0.f < 0) return;
  const int r0 = t0.r0, L = t0.L;
  const int nkc = ((L + 31) & ~31) >> 5;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  TileDesc t = t0;
  t.rb = t0.rb * MS + kw;
  const bool act = t.rb < ((L + 15) >> 4);
  const v8bf* zb = reinterpret_cast<const v8bf*>(a.zero);
  const v8bf* P = reinterpret_cast<const v8bf*>(reinterpret_cast<const char*>(a.P) + t.poff) +
                  (int64_t)(act ? t.rb : 0) * nkc * 6 * 64 + lane;
  int wc[NB];
  bool wok[NB];
  tile_cols<NB>(a, t, li, wc, wok);
  const int c = threadIdx.x % CW, rr0 = threadIdx.x / CW;
  int sw;
  bool sok;
  {
    const int nc = a.cols ? a.ncols[t.f] : a.W;
    const int sl = t.wb * CW + c;
    sok = sl < nc;
    sw = a.cols ? (sok ? a.cols[(int64_t)t.f * a.W + sl] : 0) : sl;
  }
  const double2* zx = reinterpret_cast<const double2*>(a.zero);
  v4f rr[NB], ii[NB], ri[NB], ir[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) rr[nb] = ii[nb] = ri[nb] = ir[nb] = (v4f){0.f, 0.f, 0.f, 0.f};
  double2 sv[PER];
  // State operands of chunk kc (rows past the fibre read the zero buffer).  The offset is
  // computed unconditionally and pinned by an empty asm operand, so the pointer select stays a
  // select: a load under a branch makes the compiler wait for every outstanding load at the
  // join, including the next chunk's prefetch.  (Pinning the pointer itself would lose its
  // address space and turn the loads into flat loads, which LDS waits also wait for.)
  auto load_state = [&](int kc) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int k = 32 * kc + rr0 + j * RSTEP;
      const bool ok = sok && k < L;
      int64_t off = xrow<GATHER>(a, r0 + (ok ? k : 0)) * a.W + sw;
      asm volatile("" : "+v"(off));
      sv[j] = *(ok ? a.X + off : zx);
    }
  };
  // fp32(x) split exactly into three bf16 terms, six planes [term re/im][column][k]
  auto store_state = [&](int buf) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      unsigned short q0, q1, q2, q3, q4, q5;
      split3x((float)sv[j].x, q0, q1, q2);
      split3x((float)sv[j].y, q3, q4, q5);
      const int k = rr0 + j * RSTEP;
      xb[buf][0][c][k] = q0;
      xb[buf][1][c][k] = q1;
      xb[buf][2][c][k] = q2;
      xb[buf][3][c][k] = q3;
      xb[buf][4][c][k] = q4;
      xb[buf][5][c][k] = q5;
    }
  };
  // the tile's band of chunks [klo, khi), and this wave's own [wlo, whi) inside it (its row
  // block's band; the staged chunks cover the union)
  int klo, khi;
  tile_band(t0, 32 * nkc, 32, klo, khi);
  int wlo = klo, whi = khi;
  if (a.rb_band && t0.bb >= 0 && act) {
    const int2 wb = reinterpret_cast<const int2*>(a.rb_band)[t0.bb + t.rb];
    wlo = wb.x / 32;
    whi = (min(wb.y, 32 * nkc) + 31) / 32;
  }
  auto mine = [&](int kc) { return act && kc >= wlo && kc < whi; };
  // this wave's propagator planes of chunk kc (E re/im terms 0..2), zeros outside its band
  auto load_e = [&](v8bf (&E)[6], int kc) {
    const bool in = mine(kc);
#pragma unroll
    for (int pl = 0; pl < 6; ++pl) {
      int64_t off = ((int64_t)kc * 6 + pl) * 64;
      asm volatile("" : "+v"(off));
      E[pl] = *(in ? P + off : zb);
    }
  };
  auto mma = [&](const v8bf (&E)[6], int buf) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      // one column block's operands at a time (keeps the next block's LDS reads from being
      // hoisted, which would hold twice the registers)
      if (nb > 0) __builtin_amdgcn_sched_barrier(0);
      const int col = nb * 16 + li;
      const v8bf Xr0 = *reinterpret_cast<const v8bf*>(&xb[buf][0][col][8 * lk]);
      const v8bf Xr1 = *reinterpret_cast<const v8bf*>(&xb[buf][1][col][8 * lk]);
      const v8bf Xr2 = *reinterpret_cast<const v8bf*>(&xb[buf][2][col][8 * lk]);
      const v8bf Xi0 = *reinterpret_cast<const v8bf*>(&xb[buf][3][col][8 * lk]);
      const v8bf Xi1 = *reinterpret_cast<const v8bf*>(&xb[buf][4][col][8 * lk]);
      const v8bf Xi2 = *reinterpret_cast<const v8bf*>(&xb[buf][5][col][8 * lk]);
      rr[nb] = mma3(rr[nb], E[0], E[2], E[4], Xr0, Xr1, Xr2);
      ii[nb] = mma3(ii[nb], E[1], E[3], E[5], Xi0, Xi1, Xi2);
      ri[nb] = mma3(ri[nb], E[0], E[2], E[4], Xi0, Xi1, Xi2);
      ir[nb] = mma3(ir[nb], E[1], E[3], E[5], Xr0, Xr1, Xr2);
    }
  };
  // Ping-pong operand buffers over pairs of chunks: chunk kc multiplies EA (or EB) while the
  // next chunk's state values and planes load into sv and EB (or EA); no register copies.
  v8bf EA[6], EB[6];
  load_state(klo);
  load_e(EA, klo);
  store_state(0);
  __syncthreads();
  for (int kc = klo; kc < khi; kc += 2) {
    load_state(kc + 1);
    load_e(EB, kc + 1);
    __builtin_amdgcn_sched_barrier(0);
    if (mine(kc)) mma(EA, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (kc + 1 >= khi) break;
    store_state(1);
    __syncthreads();
    load_state(kc + 2);
    load_e(EA, kc + 2);
    __builtin_amdgcn_sched_barrier(0);
    if (mine(kc + 1)) mma(EB, 1);
    __builtin_amdgcn_sched_barrier(0);
    if (kc + 2 >= khi) break;
    store_state(0);
    __syncthreads();
  }
  if (!act) return;
  double acc[NB][2][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[nb][0][r] = (double)rr[nb][r] - (double)ii[nb][r];
      acc[nb][1][r] = (double)ri[nb][r] + (double)ir[nb][r];
    }
  pass_epilogue<NB, 1, true, false>(a, t, acc, nullptr, wc, wok);
}

// ---------------------------------------------------------------- single-state fibre pass (W = 1)
// y += p x and (sr, si) <- h (sr, si) for complex operands as explicit fused multiply-adds in
// a fixed order, so the per-fibre and the orbit single-state kernels round alike
__device__ __forceinline__ void cmac(double& yr, double& yi, double pr, double pi, double2 x) {
  yr = __builtin_fma(pr, x.x, yr);
  yr = __builtin_fma(-pi, x.y, yr);
  yi = __builtin_fma(pr, x.y, yi);
  yi = __builtin_fma(pi, x.x, yi);
}
__device__ __forceinline__ void cscale(double& sr, double& si, double2 h) {
  const double zr = __builtin_fma(h.x, sr, -(h.y * si));
  si = __builtin_fma(h.x, si, h.y * sr);
  sr = zr;
}
// Single-state GEMV, one 16-row block per tile: each propagator entry is read once per pass.
// Lane (li, lk) of chunk (rb, k) multiplies entry (16rb+li, col) by x[col]; the four k-lanes
// and the KS waves are summed in fixed order.  Mixed formats: E entries (rounded to their
// storage precision) times the FP64 state, FP64 accumulation, plus the FP64 diagonal term.
template <int KS, int FMT, bool BATCH>
__device__ __forceinline__ void k_gemv_tile(const PassArgs& a0, int ti, double* red) {
  const TileDesc t = a0.tiles[ti];
  if (t.f < 0) return;
  const PassArgs a = BATCH ? a0.batch[t.f] : a0;
  const int r0 = t.r0, L = t.L;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const char* Pb = reinterpret_cast<const char*>(a.P) + t.poff;
  double yr = 0.0, yi = 0.0;
  if constexpr (FMT == PF_BF16X3) {
    const int nkc = ((L + 31) & ~31) >> 5;
    const v8u16* P = reinterpret_cast<const v8u16*>(Pb) + (int64_t)t.rb * nkc * 6 * 64 + lane;
    int klo, khi;
    tile_band(t, 32 * nkc, 32, klo, khi);
    for (int kc = klo + kw; kc < khi; kc += KS) {
      const v8u16* Pc = P + (int64_t)kc * 6 * 64;
      const v8u16 r0v = Pc[0], i0v = Pc[64], r1v = Pc[128], i1v = Pc[192], r2v = Pc[256], i2v = Pc[320];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kc + 8 * lk + e;
        if (k < L) {
          const double2 x = a.X[in_row(a, r0 + k)];
          const double er = (double)(bf2f(r0v[e]) + bf2f(r1v[e]) + bf2f(r2v[e]));
          const double ei = (double)(bf2f(i0v[e]) + bf2f(i1v[e]) + bf2f(i2v[e]));
          cmac(yr, yi, er, ei, x);
        }
      }
    }
  } else {
    // Groups of G k-steps: all loads of a group are issued before its products, with the
    // state operand of positions past the fibre read from the zero buffer (their propagator
    // entries are zero padding), so the loads stay branch-free; the products are summed in
    // k-step order as one at a time.
    using PT = typename std::conditional<FMT == PF_F64, double2, float2>::type;
    constexpr int G = 8;
    const int nks = ((L + 15) & ~15) >> 2;
    const double2* zx = reinterpret_cast<const double2*>(a.zero);
    const PT* P = reinterpret_cast<const PT*>(Pb) + (int64_t)t.rb * nks * 64 + lane;
    int klo, khi;
    tile_band(t, 4 * nks, 4, klo, khi);
    int ks = klo + kw;
    for (; ks + (G - 1) * KS < khi; ks += G * KS) {
      PT p[G];
      double2 x[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int kk = ks + g * KS, k = 4 * kk + lk;
        const bool ok = k < L;
        p[g] = P[(int64_t)kk * 64];
        x[g] = *(ok ? a.X + in_row(a, r0 + (ok ? k : 0)) : zx);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) cmac(yr, yi, p[g].x, p[g].y, x[g]);
    }
    for (; ks < khi; ks += KS) {
      const int k = 4 * ks + lk;
      const bool ok = k < L;
      const double2 x = *(ok ? a.X + in_row(a, r0 + (ok ? k : 0)) : zx);
      const PT pe = P[(int64_t)ks * 64];
      cmac(yr, yi, pe.x, pe.y, x);
    }
  }
  // sum the four k-lanes of each row (lanes li, li+16, li+32, li+48)
  yr += __shfl_xor(yr, 16);
  yi += __shfl_xor(yi, 16);
  yr += __shfl_xor(yr, 32);
  yi += __shfl_xor(yi, 32);
  if (lk == 0) {
    red[(kw * 2 + 0) * 16 + li] = yr;
    red[(kw * 2 + 1) * 16 + li] = yi;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int lr = threadIdx.x;
    const int arow = 16 * t.rb + lr;
    if (arow < L) {
      double sr = 0.0, si = 0.0;
      for (int w = 0; w < KS; ++w) {
        sr += red[(w * 2 + 0) * 16 + lr];
        si += red[(w * 2 + 1) * 16 + lr];
      }
      const int p = r0 + arow;
      if (FMT != PF_F64 || a.wt) {
        const double2 x = a.X[in_row(a, p)];
        if (FMT != PF_F64) {
          const double2 dg = a.diag[t.d0 + arow];
          cmac(sr, si, dg.x, dg.y, x);
        }
        if (a.wt) {
          const double g = a.wt[t.f];
          sr = x.x + g * (sr - x.x);
          si = x.y + g * (si - x.y);
        }
      }
      if (a.ph) cscale(sr, si, a.ph[a.ph_idx ? a.ph_idx[p] : p]);
      a.Y[a.out_pos ? a.out_pos[p] : p] = make_double2(sr, si);
    }
  }
}

template <int KS, int FMT, bool BATCH>
__global__ __launch_bounds__(64 * KS) void k_gemv(PassArgs a0) {
  __shared__ double red[2 * KS * 16];
  if (a0.tcount && (int)blockIdx.x >= *a0.tcount) return;
  k_gemv_tile<KS, FMT, BATCH>(a0, blockIdx.x, red);
}

template <int KS, int FMT>
__global__ __launch_bounds__(64 * KS) void k_gemv_persist(PassArgs a0) {
  __shared__ double red[2 * KS * 16];
  persistent_tiles(a0, [&](int ti) { k_gemv_tile<KS, FMT, true>(a0, ti, red); });
}

// ---------------------------------------------------------------- single-state orbit pass (W = 1)
// Fibres with one stored propagator (point-symmetry orbits, kappa = 1 translation classes)
// are multiplied together: a tile covers a 16-row block of the shared propagator for the
// states of up to M fibres of a group (PassArgs::orbit), so every propagator chunk is loaded
// once for the whole group instead of once per fibre.  Each fibre's products are summed in
// the order k_gemv_tile sums them for the same KS (k-steps in order per lane, then the four
// k-lanes, then the waves), so the two kernels give identical results.
template <int KS, int FMT, int M>
__global__ __launch_bounds__(64 * KS) void k_gemv_orbit(PassArgs a) {
  __shared__ double red[KS * M * 2 * 16];
  const TileDesc t = a.tiles[blockIdx.x];
  if (t.f < 0) return;
  const int32_t* og = a.orbit + (int64_t)t.f * kOrbitStride;
  const int nm = og[0];
  int r0[M];
#pragma unroll
  for (int m = 0; m < M; ++m) r0[m] = og[1 + m];
  const int L = t.L;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const char* Pb = reinterpret_cast<const char*>(a.P) + t.poff;
  double yr[M], yi[M];
#pragma unroll
  for (int m = 0; m < M; ++m) yr[m] = yi[m] = 0.0;
  if constexpr (FMT == PF_BF16X3) {
    const int nkc = ((L + 31) & ~31) >> 5;
    const v8u16* P = reinterpret_cast<const v8u16*>(Pb) + (int64_t)t.rb * nkc * 6 * 64 + lane;
    int klo, khi;
    tile_band(t, 32 * nkc, 32, klo, khi);
    for (int kc = klo + kw; kc < khi; kc += KS) {
      const v8u16* Pc = P + (int64_t)kc * 6 * 64;
      const v8u16 r0v = Pc[0], i0v = Pc[64], r1v = Pc[128], i1v = Pc[192], r2v = Pc[256], i2v = Pc[320];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kc + 8 * lk + e;
        if (k < L) {
          const double er = (double)(bf2f(r0v[e]) + bf2f(r1v[e]) + bf2f(r2v[e]));
          const double ei = (double)(bf2f(i0v[e]) + bf2f(i1v[e]) + bf2f(i2v[e]));
#pragma unroll
          for (int m = 0; m < M; ++m) {
            const double2 x = a.X[in_row(a, r0[m] + k)];
            cmac(yr[m], yi[m], er, ei, x);
          }
        }
      }
    }
  } else {
    // groups of G k-steps, every load of a group issued before its products (state operands
    // past the fibre read the zero buffer, as in k_gemv_tile)
    using PT = typename std::conditional<FMT == PF_F64, double2, float2>::type;
    constexpr int G = M <= 2 ? 4 : (M <= 4 ? 2 : 1);
    const int nks = ((L + 15) & ~15) >> 2;
    const double2* zx = reinterpret_cast<const double2*>(a.zero);
    const PT* P = reinterpret_cast<const PT*>(Pb) + (int64_t)t.rb * nks * 64 + lane;
    int klo, khi;
    tile_band(t, 4 * nks, 4, klo, khi);
    int ks = klo + kw;
    for (; ks + (G - 1) * KS < khi; ks += G * KS) {
      PT p[G];
      double2 x[G][M];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int kk = ks + g * KS, k = 4 * kk + lk;
        const bool ok = k < L;
        p[g] = P[(int64_t)kk * 64];
#pragma unroll
        for (int m = 0; m < M; ++m) x[g][m] = *(ok ? a.X + in_row(a, r0[m] + (ok ? k : 0)) : zx);
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int m = 0; m < M; ++m) cmac(yr[m], yi[m], p[g].x, p[g].y, x[g][m]);
    }
    for (; ks < khi; ks += KS) {
      const int k = 4 * ks + lk;
      const bool ok = k < L;
      double2 x[M];
#pragma unroll
      for (int m = 0; m < M; ++m) x[m] = *(ok ? a.X + in_row(a, r0[m] + (ok ? k : 0)) : zx);
      const PT pe = P[(int64_t)ks * 64];
#pragma unroll
      for (int m = 0; m < M; ++m) cmac(yr[m], yi[m], pe.x, pe.y, x[m]);
    }
  }
  // sum the four k-lanes of each row, then the waves in order
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double vr = yr[m], vi = yi[m];
    vr += __shfl_xor(vr, 16);
    vi += __shfl_xor(vi, 16);
    vr += __shfl_xor(vr, 32);
    vi += __shfl_xor(vi, 32);
    if (lk == 0) {
      red[((kw * M + m) * 2 + 0) * 16 + li] = vr;
      red[((kw * M + m) * 2 + 1) * 16 + li] = vi;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 16 * M; idx += 64 * KS) {
    const int lr = idx & 15, m = idx >> 4;
    const int arow = 16 * t.rb + lr;
    if (m >= nm || arow >= L) continue;
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < KS; ++w) {
      sr += red[((w * M + m) * 2 + 0) * 16 + lr];
      si += red[((w * M + m) * 2 + 1) * 16 + lr];
    }
    const int p = og[1 + m] + arow;
    if (FMT != PF_F64) {
      const double2 x = a.X[in_row(a, p)];
      const double2 dg = a.diag[t.d0 + arow];
      cmac(sr, si, dg.x, dg.y, x);
    }
    if (a.ph) cscale(sr, si, a.ph[a.ph_idx ? a.ph_idx[p] : p]);
    a.Y[a.out_pos ? a.out_pos[p] : p] = make_double2(sr, si);
  }
}

// ---------------------------------------------------------------- single-state passes, one row per lane
// A wave covers four 16-row blocks of a propagator (lane l: block l / 16 of the tile, row
// l % 16) and reads, for each k-step, all columns of its row from the lane slots of the
// stored chunk (four slots of one column for FP64 / FP32, four slots of eight columns for
// BF16x3), so the state operand of a k-step is the same for the whole wave: it is read once
// per wave through the scalar cache instead of once per lane.  ORB: the tile
// multiplies up to M fibres of a group with one propagator (PassArgs::orbit), else the tile's
// own fibre.  Per fibre and row the products are summed in column order, then the KS waves in
// order, so orbit and per-fibre tiles give identical results.  The k-steps run over the union
// of the four blocks' bands, and each block's lanes take zeros outside their own block's band.
template <int KS, int FMT, int M, bool ORB, bool GATHER>
__global__ __launch_bounds__(64 * KS) void k_gemv_rows(PassArgs a) {
  static_assert(ORB || M == 1, "a per-fibre tile has one fibre");
  __shared__ double red[KS * M * 2 * 64];
  const TileDesc t = a.tiles[blockIdx.x];
  if (t.f < 0) return;
  int nm = 1, r0[M];
  if constexpr (ORB) {
    const int32_t* og = a.orbit + (int64_t)t.f * kOrbitStride;
    nm = og[0];
#pragma unroll
    for (int m = 0; m < M; ++m) r0[m] = og[1 + m];
  } else {
    r0[0] = t.r0;
  }
  const int L = t.L;
  const int lane = threadIdx.x & 63, kw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, q = lane >> 4;
  const int nrb = (L + 15) >> 4;
  const int rbq = 4 * t.rb + q;
  const bool rowok = rbq < nrb;
  const char* Pb = reinterpret_cast<const char*>(a.P) + t.poff;
  // each row block's own band (fibre positions): its lanes read the zero buffer outside it
  int qlo = 0, qhi = kBandEnd;
  if (a.rb_band && t.bb >= 0 && rowok) {
    const int2 b = reinterpret_cast<const int2*>(a.rb_band)[t.bb + rbq];
    qlo = b.x;
    qhi = b.y;
  }
  double yr[M], yi[M];
#pragma unroll
  for (int m = 0; m < M; ++m) yr[m] = yi[m] = 0.0;
  if constexpr (FMT == PF_BF16X3) {
    // BF16x3 chunks of 32 columns: the row's four lane slots hold 8 consecutive columns each
    // (six planes of 8 bf16 per slot); per slot, the state operand is 8 consecutive rows of
    // every fibre (two 64-byte reads where contiguous)
    const int nkc = ((L + 31) & ~31) >> 5;
    const v8u16* zp = reinterpret_cast<const v8u16*>(a.zero);
    const v8u16* Pq = reinterpret_cast<const v8u16*>(Pb) + (int64_t)(rowok ? rbq : 0) * nkc * 6 * 64 + li;
    int klo, khi;
    tile_band(t, 32 * nkc, 32, klo, khi);
    struct X8 {
      double2 v[8];
    };
    for (int kc = klo + kw; kc < khi; kc += KS) {
      const bool in = rowok && 32 * kc >= qlo && 32 * kc < qhi;
      const v8u16* Pc = Pq + (int64_t)kc * 6 * 64;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v8u16 pl[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) pl[k] = *(in ? Pc + 64 * k + 16 * j : zp);
        double er[8], ei[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          er[e] = (double)(bf2f(pl[0][e]) + bf2f(pl[2][e]) + bf2f(pl[4][e]));
          ei[e] = (double)(bf2f(pl[1][e]) + bf2f(pl[3][e]) + bf2f(pl[5][e]));
        }
        const int c0 = 32 * kc + 8 * j;
        if (!GATHER && c0 + 7 < L) {
#pragma unroll
          for (int m = 0; m < M; ++m) {
            const X8 x = *reinterpret_cast<const X8*>(a.X + r0[m] + c0);
#pragma unroll
            for (int e = 0; e < 8; ++e) cmac(yr[m], yi[m], er[e], ei[e], x.v[e]);
          }
        } else {
#pragma unroll
          for (int m = 0; m < M; ++m)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const double2 x = a.X[xrow<GATHER>(a, r0[m] + min(c0 + e, L - 1))];
              cmac(yr[m], yi[m], er[e], ei[e], x);
            }
        }
      }
    }
  } else {
    using PT = typename std::conditional<FMT == PF_F64, double2, float2>::type;
    const int nks = ((L + 15) & ~15) >> 2;
    const PT* zp = reinterpret_cast<const PT*>(a.zero);
    const PT* Pq = reinterpret_cast<const PT*>(Pb) + (int64_t)(rowok ? rbq : 0) * nks * 64 + li;
    int klo, khi;
    tile_band(t, 4 * nks, 4, klo, khi);
    auto src = [&](int kk, int c) { return (rowok && 4 * kk >= qlo && 4 * kk < qhi) ? Pq + (int64_t)kk * 64 + 16 * c : zp; };
    // The state operand of a k-step: four consecutive rows of every fibre, one 64-byte read per
    // fibre where its rows are contiguous (no gather, k-step inside the fibre); columns past the
    // fibre multiply zero padding and read the fibre's last row instead.  One k-step's loads in
    // flight per wave (two measured slower: fewer waves fit).
    struct X4 {
      double2 v[4];
    };
    for (int kk = klo + kw; kk < khi; kk += KS) {
      PT e[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) e[c] = *src(kk, c);
      if (!GATHER && 4 * kk + 3 < L) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const X4 x = *reinterpret_cast<const X4*>(a.X + r0[m] + 4 * kk);
#pragma unroll
          for (int c = 0; c < 4; ++c) cmac(yr[m], yi[m], e[c].x, e[c].y, x.v[c]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double2 x = a.X[xrow<GATHER>(a, r0[m] + min(4 * kk + c, L - 1))];
            cmac(yr[m], yi[m], e[c].x, e[c].y, x);
          }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    red[((kw * M + m) * 2 + 0) * 64 + lane] = yr[m];
    red[((kw * M + m) * 2 + 1) * 64 + lane] = yi[m];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * M; idx += 64 * KS) {
    const int ln = idx & 63, m = idx >> 6;
    const int arow = 16 * (4 * t.rb + (ln >> 4)) + (ln & 15);
    if (m >= nm || arow >= L) continue;
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < KS; ++w) {
      sr += red[((w * M + m) * 2 + 0) * 64 + ln];
      si += red[((w * M + m) * 2 + 1) * 64 + ln];
    }
    const int p = (ORB ? a.orbit[(int64_t)t.f * kOrbitStride + 1 + m] : t.r0) + arow;
    if (FMT != PF_F64) {
      const double2 x = a.X[in_row(a, p)];
      const double2 dg = a.diag[t.d0 + arow];
      cmac(sr, si, dg.x, dg.y, x);
    }
    if (a.ph) cscale(sr, si, a.ph[a.ph_idx ? a.ph_idx[p] : p]);
    a.Y[a.out_pos ? a.out_pos[p] : p] = make_double2(sr, si);
  }
}

// ---------------------------------------------------------------- FP64 reductions
// kind 0: |c|^2;  kind 1: 1/2 K2 |c|^2 + Re conj(c_iw) sum_p v_p c_{nbr(i,p), w} (both layers)
__global__ __launch_bounds__(256) void k_reduce_partial(int kind, int64_t N, int W, const double2* c,
                                                        const double* K2, int nv1, const int32_t* nbr1,
                                                        const double2* v1, int nv2, const int32_t* nbr2,
                                                        const double2* v2, int nv3, const int32_t* nbr3,
                                                        const double2* v3, double* partial, int R) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * R;
  const int64_t i1 = min(N, i0 + R);
  const int WB = W < 256 ? W : 256;
  const int S = 256 / WB;
  const int tid = threadIdx.x;
  for (int w0 = 0; w0 < W; w0 += WB) {
    const int w = w0 + tid % WB, s = tid / WB;
    double acc = 0.0;
    if (w < W && s < S) {
      for (int64_t i = i0 + s; i < i1; i += S) {
        const double2 x = c[i * W + w];
        const double m2 = x.x * x.x + x.y * x.y;
        if (kind == 0) {
          acc += m2;
        } else {
          double hr = 0.0, hi = 0.0;
          for (int p = 0; p < nv1; ++p) {
            const int j = nbr1[i * nv1 + p];
            if (j >= 0) {
              const double2 y = c[(int64_t)j * W + w], v = v1[p];
              hr += v.x * y.x - v.y * y.y;
              hi += v.x * y.y + v.y * y.x;
            }
          }
          for (int p = 0; p < nv2; ++p) {
            const int j = nbr2[i * nv2 + p];
            if (j >= 0) {
              const double2 y = c[(int64_t)j * W + w], v = v2[p];
              hr += v.x * y.x - v.y * y.y;
              hi += v.x * y.y + v.y * y.x;
            }
          }
          for (int p = 0; p < nv3; ++p) {
            const int j = nbr3[i * nv3 + p];
            if (j >= 0) {
              const double2 y = c[(int64_t)j * W + w], v = v3[p];
              hr += v.x * y.x - v.y * y.y;
              hi += v.x * y.y + v.y * y.x;
            }
          }
          acc += 0.5 * K2[i] * m2 + (x.x * hr + x.y * hi);
        }
      }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < WB && w0 + tid < W) {
      double sum = 0.0;
      for (int j = 0; j < S; ++j) sum += red[j * WB + tid];
      partial[(int64_t)b * W + w0 + tid] = sum;
    }
    __syncthreads();
  }
}

__global__ void k_reduce_final(int nblocks, int W, const double* partial, double* out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < W) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * W + w];
    out[w] = s;
  }
}

__global__ __launch_bounds__(256) void k_fibre_mass(const int32_t* ptr, const int32_t* rows, int W,
                                                    const double2* c, double* out) {
  __shared__ double red[256];
  const int f = blockIdx.x;
  const int r0 = ptr[f], L = ptr[f + 1] - r0;
  const int WB = W < 256 ? W : 256;
  const int S = 256 / WB;
  const int tid = threadIdx.x;
  for (int w0 = 0; w0 < W; w0 += WB) {
    const int w = w0 + tid % WB, s = tid / WB;
    // four independent partial sums keep four rows in flight per thread
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    if (w < W && s < S) {
      int a = s;
      for (; a + 3 * S < L; a += 4 * S) {
        const double2 x0 = c[(int64_t)rows[r0 + a] * W + w];
        const double2 x1 = c[(int64_t)rows[r0 + a + S] * W + w];
        const double2 x2 = c[(int64_t)rows[r0 + a + 2 * S] * W + w];
        const double2 x3 = c[(int64_t)rows[r0 + a + 3 * S] * W + w];
        acc0 += x0.x * x0.x + x0.y * x0.y;
        acc1 += x1.x * x1.x + x1.y * x1.y;
        acc2 += x2.x * x2.x + x2.y * x2.y;
        acc3 += x3.x * x3.x + x3.y * x3.y;
      }
      for (; a < L; a += S) {
        const double2 x = c[(int64_t)rows[r0 + a] * W + w];
        acc0 += x.x * x.x + x.y * x.y;
      }
    }
    red[tid] = (acc0 + acc1) + (acc2 + acc3);
    __syncthreads();
    if (tid < WB && w0 + tid < W) {
      double sum = 0.0;
      for (int j = 0; j < S; ++j) sum += red[j * WB + tid];
      out[(int64_t)f * W + w0 + tid] = sum;
    }
    __syncthreads();
  }
}

// ================================================================ launchers
hipError_t launch_assemble(hipStream_t s, int nb, const int32_t* fid, const int32_t* ptr, const int32_t* rows,
                           const int32_t* mn, int d, int stride, int own, double kfac, const double* K2, int nv,
                           const int32_t* vidx, const double* vre, const double* vim, int embed, double* A,
                           const int64_t* moff, const int32_t* ndim) {
  hipLaunchKernelGGL(k_assemble, dim3(nb), dim3(256), 0, s, fid, ptr, rows, mn, d, stride, own, kfac, K2, nv, vidx,
                     vre, vim, embed, A, moff, ndim);
  return hipGetLastError();
}

hipError_t launch_jacobi(hipStream_t s, int nf, int maxn, double* A, double* VT, const int64_t* moff,
                         const int32_t* ndim, double* lam, const int64_t* loff, int32_t* info, int maxsweeps,
                         const int32_t* sel) {
  if (nf == 0) return hipSuccess;
  const size_t shm = (size_t)(maxn / 2) * (2 * sizeof(double) + 2 * sizeof(int));
  if (maxn > 256)
    hipLaunchKernelGGL(k_jacobi<1024>, dim3(nf), dim3(1024), shm, s, A, VT, moff, ndim, lam, loff, info,
                       maxsweeps, sel);
  else
    hipLaunchKernelGGL(k_jacobi<256>, dim3(nf), dim3(256), shm, s, A, VT, moff, ndim, lam, loff, info,
                       maxsweeps, sel);
  return hipGetLastError();
}

hipError_t launch_eig_fn(hipStream_t s, int64_t nlam, const double* lam, double t, int flow, double2* gh) {
  if (nlam == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eig_fn, dim3((unsigned)((nlam + 255) / 256)), dim3(256), 0, s, nlam, lam, t, flow, gh);
  return hipGetLastError();
}

hipError_t launch_band(hipStream_t s, int fmt, int nb, const int32_t* fid, const int32_t* ptr, const void* P,
                       const int64_t* poff, const int64_t* boff, double tol, int32_t* band) {
  if (nb == 0) return hipSuccess;
  if (fmt == PF_F64)
    hipLaunchKernelGGL(k_band<PF_F64>, dim3(nb), dim3(256), 0, s, fid, ptr, P, poff, boff, tol, band);
  else if (fmt == PF_F32)
    hipLaunchKernelGGL(k_band<PF_F32>, dim3(nb), dim3(256), 0, s, fid, ptr, P, poff, boff, tol, band);
  else
    hipLaunchKernelGGL(k_band<PF_BF16X3>, dim3(nb), dim3(256), 0, s, fid, ptr, P, poff, boff, tol, band);
  return hipGetLastError();
}

hipError_t launch_form(hipStream_t s, int fmt, int nb, int maxL, const int32_t* fid, const int32_t* ptr,
                       const double* VT, const int64_t* moff, const int32_t* ndim, const int32_t* embed,
                       const double2* gh, const int64_t* loff, void* P, const int64_t* poff, double2* diag) {
  const int64_t maxLL = (int64_t)maxL * maxL;
  const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>((maxLL + 255) / 256, 4096));
  const dim3 g(nb, gy);
  if (fmt == PF_F64)
    hipLaunchKernelGGL(k_form<PF_F64>, g, dim3(256), 0, s, fid, ptr, VT, moff, ndim, embed, gh, loff, P, poff, diag);
  else if (fmt == PF_F32)
    hipLaunchKernelGGL(k_form<PF_F32>, g, dim3(256), 0, s, fid, ptr, VT, moff, ndim, embed, gh, loff, P, poff, diag);
  else
    hipLaunchKernelGGL(k_form<PF_BF16X3>, g, dim3(256), 0, s, fid, ptr, VT, moff, ndim, embed, gh, loff, P, poff,
                       diag);
  return hipGetLastError();
}

hipError_t launch_phase_table(hipStream_t s, int64_t N, const double* K2, double scale, double2* ph) {
  hipLaunchKernelGGL(k_phase_table, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, K2, scale, ph);
  return hipGetLastError();
}

hipError_t launch_phase_apply(hipStream_t s, int64_t N, int W, const double2* ph, double2* c) {
  int TW = 1;
  while (TW < W && TW < 256) TW <<= 1;
  const int64_t rows_per_block = 256 / TW;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + rows_per_block - 1) / rows_per_block,
                                                                        256 * 64));
  hipLaunchKernelGGL(k_phase_apply, dim3(grid), dim3(256), 0, s, N, W, TW, ph, c);
  return hipGetLastError();
}

// Prefetch depth of the FP64/FP32 passes (k-steps per register group); LSX_PREFETCH
// selects 1, 2 or 4 (default 2).
static int prefetch_depth() {
  static int u = [] {
    const char* v = std::getenv("LSX_PREFETCH");
    const int x = v ? std::atoi(v) : 2;
    return (x == 1 || x == 4) ? x : 2;
  }();
  return u;
}

// Set while prepare_persistent() runs: persistent launchers compute their grid (and so query
// the kernel's occupancy) and return without launching.
static thread_local bool g_prepare_only = false;

// Grid of a persistent launch: the kernel's resident workgroups per CU times the CU count,
// rounded down to a multiple of 8 (whole XCD rounds), at most the tile count rounded up to 8.
// The occupancy of each kernel is queried once.
static unsigned persistent_grid(const void* fn, int threads, size_t shm, int ntiles) {
  static std::map<const void*, int> cap;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cap.find(fn);
  if (it == cap.end()) {
    int dev = 0, ncu = 256, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, shm) != hipSuccess || per < 1) per = 1;
    it = cap.emplace(fn, std::max(8, (per * ncu) / 8 * 8)).first;
  }
  const int want = (ntiles + 7) / 8 * 8;
  return (unsigned)std::max(8, std::min(want, it->second));
}

template <int NB, int KS, int U, bool G>
static hipError_t launch_mfma_persist(hipStream_t s, int fmt, int ntiles, const PassArgs& a0) {
  PassArgs a = a0;
  a.ntiles = ntiles;
  const size_t shm = KS > 1 ? (size_t)KS * NB * 2 * 4 * 64 * sizeof(double) : 0;
  const void* fn = fmt == PF_F64   ? reinterpret_cast<const void*>(&k_pass_f64_persist<NB, KS, U, G>)
                   : fmt == PF_F32 ? reinterpret_cast<const void*>(&k_pass_f32_persist<NB, KS, U, G>)
                                   : reinterpret_cast<const void*>(&k_pass_bf16x3_persist<NB, KS, 1, G>);
  const dim3 grid(persistent_grid(fn, 64 * KS, shm, ntiles));
  if (g_prepare_only) return hipSuccess;
  if (fmt == PF_F64)
    hipLaunchKernelGGL((k_pass_f64_persist<NB, KS, U, G>), grid, dim3(64 * KS), shm, s, a);
  else if (fmt == PF_F32)
    hipLaunchKernelGGL((k_pass_f32_persist<NB, KS, U, G>), grid, dim3(64 * KS), shm, s, a);
  else
    hipLaunchKernelGGL((k_pass_bf16x3_persist<NB, KS, 1, G>), grid, dim3(64 * KS), shm, s, a);
  return hipGetLastError();
}

template <int NB, int KS, int U, bool G, bool B>
static hipError_t launch_mfma_u(hipStream_t s, int fmt, int ntiles, const PassArgs& a) {
  const size_t shm = KS > 1 ? (size_t)KS * NB * 2 * 4 * 64 * sizeof(double) : 0;
  if constexpr (B) {
    if (a.persist) return launch_mfma_persist<NB, KS, U, G>(s, fmt, ntiles, a);
  }
  if (fmt == PF_F64)
    hipLaunchKernelGGL((k_pass_f64<NB, KS, U, G, B>), dim3(ntiles), dim3(64 * KS), shm, s, a);
  else if (fmt == PF_F32)
    hipLaunchKernelGGL((k_pass_f32<NB, KS, U, G, B>), dim3(ntiles), dim3(64 * KS), shm, s, a);
  else
    hipLaunchKernelGGL((k_pass_bf16x3<NB, KS, 1, G, B>), dim3(ntiles), dim3(64 * KS), shm, s, a);
  return hipGetLastError();
}

template <int NB, int KS, bool G>
static hipError_t launch_mfma_g(hipStream_t s, int fmt, int ntiles, const PassArgs& a, bool batched) {
  if (batched)
    return (fmt != PF_BF16X3 && a.u == 1) ? launch_mfma_u<NB, KS, 1, G, true>(s, fmt, ntiles, a)
                                          : launch_mfma_u<NB, KS, 2, G, true>(s, fmt, ntiles, a);
  switch (fmt == PF_BF16X3 ? 1 : (a.u == 1 || a.u == 2 || a.u == 4) ? a.u : prefetch_depth()) {
    case 1: return launch_mfma_u<NB, KS, 1, G, false>(s, fmt, ntiles, a);
    case 4: return launch_mfma_u<NB, KS, 4, G, false>(s, fmt, ntiles, a);
    default: return launch_mfma_u<NB, KS, 2, G, false>(s, fmt, ntiles, a);
  }
}

template <int NB, int KS>
static hipError_t launch_mfma(hipStream_t s, int fmt, int ntiles, const PassArgs& a, bool batched, bool gather) {
  return gather ? launch_mfma_g<NB, KS, true>(s, fmt, ntiles, a, batched)
                : launch_mfma_g<NB, KS, false>(s, fmt, ntiles, a, batched);
}

template <int KS, bool B>
static hipError_t launch_gemv(hipStream_t s, int fmt, int ntiles, const PassArgs& a0) {
  PassArgs a = a0;
  if constexpr (B) {
    if (a.persist) {
      a.ntiles = ntiles;
      const void* fn = fmt == PF_F64   ? reinterpret_cast<const void*>(&k_gemv_persist<KS, PF_F64>)
                       : fmt == PF_F32 ? reinterpret_cast<const void*>(&k_gemv_persist<KS, PF_F32>)
                                       : reinterpret_cast<const void*>(&k_gemv_persist<KS, PF_BF16X3>);
      const dim3 grid(persistent_grid(fn, 64 * KS, 0, ntiles));
      if (g_prepare_only) return hipSuccess;
      if (fmt == PF_F64)
        hipLaunchKernelGGL((k_gemv_persist<KS, PF_F64>), grid, dim3(64 * KS), 0, s, a);
      else if (fmt == PF_F32)
        hipLaunchKernelGGL((k_gemv_persist<KS, PF_F32>), grid, dim3(64 * KS), 0, s, a);
      else
        hipLaunchKernelGGL((k_gemv_persist<KS, PF_BF16X3>), grid, dim3(64 * KS), 0, s, a);
      return hipGetLastError();
    }
  }
  if (fmt == PF_F64)
    hipLaunchKernelGGL((k_gemv<KS, PF_F64, B>), dim3(ntiles), dim3(64 * KS), 0, s, a);
  else if (fmt == PF_F32)
    hipLaunchKernelGGL((k_gemv<KS, PF_F32, B>), dim3(ntiles), dim3(64 * KS), 0, s, a);
  else
    hipLaunchKernelGGL((k_gemv<KS, PF_BF16X3, B>), dim3(ntiles), dim3(64 * KS), 0, s, a);
  return hipGetLastError();
}

// single-state orbit tiles of one row block: KS waves, M the layer's largest group rounded up
// to an instantiated size
template <int KS>
static hipError_t launch_gemv_orbit_m(hipStream_t s, int fmt, int ntiles, const PassArgs& a) {
  const int gm = a.orbit_max;
#define LSX_ORBIT_M(M_)                                                                           \
  if (gm <= M_) {                                                                                 \
    if (fmt == PF_F64)                                                                            \
      hipLaunchKernelGGL((k_gemv_orbit<KS, PF_F64, M_>), dim3(ntiles), dim3(64 * KS), 0, s, a);    \
    else if (fmt == PF_F32)                                                                       \
      hipLaunchKernelGGL((k_gemv_orbit<KS, PF_F32, M_>), dim3(ntiles), dim3(64 * KS), 0, s, a);    \
    else                                                                                          \
      hipLaunchKernelGGL((k_gemv_orbit<KS, PF_BF16X3, M_>), dim3(ntiles), dim3(64 * KS), 0, s, a); \
    return hipGetLastError();                                                                     \
  }
  LSX_ORBIT_M(2)
  LSX_ORBIT_M(4)
  LSX_ORBIT_M(6)
  LSX_ORBIT_M(8)
#undef LSX_ORBIT_M
  return hipErrorInvalidValue;
}

// single-state tiles of four row blocks, one row per lane (every storage format): per-fibre
// tiles (orbit = false) or orbit tiles with M the layer's largest group rounded up
template <int KS, int FMT, int M, bool ORB>
static hipError_t launch_gemv_rows_g(hipStream_t s, int ntiles, const PassArgs& a) {
  if (a.in_pos)
    hipLaunchKernelGGL((k_gemv_rows<KS, FMT, M, ORB, true>), dim3(ntiles), dim3(64 * KS), 0, s, a);
  else
    hipLaunchKernelGGL((k_gemv_rows<KS, FMT, M, ORB, false>), dim3(ntiles), dim3(64 * KS), 0, s, a);
  return hipGetLastError();
}

template <int KS, int M, bool ORB>
static hipError_t launch_gemv_rows_m(hipStream_t s, int fmt, int ntiles, const PassArgs& a) {
  if (fmt == PF_F64) return launch_gemv_rows_g<KS, PF_F64, M, ORB>(s, ntiles, a);
  if (fmt == PF_F32) return launch_gemv_rows_g<KS, PF_F32, M, ORB>(s, ntiles, a);
  return launch_gemv_rows_g<KS, PF_BF16X3, M, ORB>(s, ntiles, a);
}

template <int KS>
static hipError_t launch_gemv_rows(hipStream_t s, int fmt, int ntiles, bool orbit, const PassArgs& a) {
  if (!orbit) return launch_gemv_rows_m<KS, 1, false>(s, fmt, ntiles, a);
  if (!a.orbit || a.orbit_max < 1 || a.orbit_max > kOrbitMax || a.wt || a.tcount) return hipErrorInvalidValue;
  const int gm = a.orbit_max;
  if (gm <= 2) return launch_gemv_rows_m<KS, 2, true>(s, fmt, ntiles, a);
  if (gm <= 4) return launch_gemv_rows_m<KS, 4, true>(s, fmt, ntiles, a);
  if (gm <= 6) return launch_gemv_rows_m<KS, 6, true>(s, fmt, ntiles, a);
  return launch_gemv_rows_m<KS, 8, true>(s, fmt, ntiles, a);
}

static hipError_t launch_gemv_orbit(hipStream_t s, int fmt, int ntiles, int ksplit, const PassArgs& a) {
  if (!a.orbit || a.orbit_max < 1 || a.orbit_max > kOrbitMax || a.wt || a.tcount) return hipErrorInvalidValue;
  switch (ksplit) {
    case 1: return launch_gemv_orbit_m<1>(s, fmt, ntiles, a);
    case 2: return launch_gemv_orbit_m<2>(s, fmt, ntiles, a);
    case 4: return launch_gemv_orbit_m<4>(s, fmt, ntiles, a);
    default: return hipErrorInvalidValue;
  }
}

// batched: tile.f is a system index into a.batch and every system has its own W; the
// caller passes gather = whether the systems' in_pos tables are set (uniform per pass)
hipError_t launch_pass(hipStream_t s, int fmt, int W, int ntiles, int nb, int ksplit, const PassArgs& a,
                       bool batched) {
  if (ntiles == 0) return hipSuccess;
  const bool gather = a.in_pos != nullptr;
  if (W == 1) {
    if (batched) return launch_gemv<4, true>(s, fmt, ntiles, a);
    if (ksplit < 0) {  // tiles of four row blocks, one row per lane, -ksplit waves
      const bool orbit = nb == kOrbitNB;
      switch (-ksplit) {
        case 1: return launch_gemv_rows<1>(s, fmt, ntiles, orbit, a);
        case 2: return launch_gemv_rows<2>(s, fmt, ntiles, orbit, a);
        case 4: return launch_gemv_rows<4>(s, fmt, ntiles, orbit, a);
        case 8: return launch_gemv_rows<8>(s, fmt, ntiles, orbit, a);
        default: return hipErrorInvalidValue;
      }
    }
    if (nb == kOrbitNB) return launch_gemv_orbit(s, fmt, ntiles, ksplit, a);
    switch (ksplit) {
      case 1: return launch_gemv<1, false>(s, fmt, ntiles, a);
      case 2: return launch_gemv<2, false>(s, fmt, ntiles, a);
      default: return launch_gemv<4, false>(s, fmt, ntiles, a);
    }
  }
  if (ksplit < 0) {
    if (batched || fmt == PF_F64) return hipErrorInvalidValue;
    if (fmt == PF_BF16X3) {
#define LSX_ROWSPLIT_BF(NB_, MS_)                                                                       \
  if (nb == NB_ && -ksplit == MS_) {                                                                    \
    if (gather)                                                                                         \
      hipLaunchKernelGGL((k_pass_bf16m<NB_, MS_, true>), dim3(ntiles), dim3(64 * MS_), 0, s, a);        \
    else                                                                                                \
      hipLaunchKernelGGL((k_pass_bf16m<NB_, MS_, false>), dim3(ntiles), dim3(64 * MS_), 0, s, a);       \
    return hipGetLastError();                                                                           \
  }
      LSX_ROWSPLIT_BF(1, 2)
      LSX_ROWSPLIT_BF(1, 4)
      LSX_ROWSPLIT_BF(1, 8)
      LSX_ROWSPLIT_BF(2, 2)
      LSX_ROWSPLIT_BF(2, 4)
      LSX_ROWSPLIT_BF(2, 8)
#undef LSX_ROWSPLIT_BF
      return hipErrorInvalidValue;
    }
#define LSX_ROWSPLIT_CASE(NB_, MS_)                                                                      \
  if (nb == NB_ && -ksplit == MS_) {                                                                    \
    if (gather)                                                                                         \
      hipLaunchKernelGGL((k_pass_f32m<NB_, MS_, true>), dim3(ntiles), dim3(64 * MS_), 0, s, a);         \
    else                                                                                                \
      hipLaunchKernelGGL((k_pass_f32m<NB_, MS_, false>), dim3(ntiles), dim3(64 * MS_), 0, s, a);        \
    return hipGetLastError();                                                                           \
  }
    LSX_ROWSPLIT_CASE(1, 2)
    LSX_ROWSPLIT_CASE(1, 4)
    LSX_ROWSPLIT_CASE(2, 2)
    LSX_ROWSPLIT_CASE(2, 4)
    LSX_ROWSPLIT_CASE(2, 8)
    LSX_ROWSPLIT_CASE(4, 2)
    LSX_ROWSPLIT_CASE(4, 4)
    LSX_ROWSPLIT_CASE(4, 8)
#undef LSX_ROWSPLIT_CASE
    return hipErrorInvalidValue;
  }
#define LSX_MFMA_CASE(NB_, KS_) \
  if (nb == NB_ && ksplit == KS_) return launch_mfma<NB_, KS_>(s, fmt, ntiles, a, batched, gather);
  LSX_MFMA_CASE(1, 1)
  LSX_MFMA_CASE(1, 2)
  LSX_MFMA_CASE(1, 4)
  LSX_MFMA_CASE(2, 1)
  LSX_MFMA_CASE(2, 2)
  LSX_MFMA_CASE(2, 4)
  LSX_MFMA_CASE(4, 1)
  LSX_MFMA_CASE(4, 2)
  LSX_MFMA_CASE(4, 4)
#undef LSX_MFMA_CASE
  return hipErrorInvalidValue;
}

hipError_t prepare_persistent(int fmt, int W, int nb, int ksplit, const PassArgs& a) {
  if (!a.persist) return hipSuccess;
  g_prepare_only = true;
  const hipError_t e = launch_pass(nullptr, fmt, W, 1, nb, ksplit, a, true);
  g_prepare_only = false;
  return e;
}

hipError_t launch_reduce(hipStream_t s, int kind, int64_t N, int W, const double2* c, const double* K2, int nv1,
                         const int32_t* nbr1, const double2* v1, int nv2, const int32_t* nbr2, const double2* v2,
                         int nv3, const int32_t* nbr3, const double2* v3, double* partial, int nblocks,
                         double* out) {
  const int R = (int)((N + nblocks - 1) / nblocks);
  hipLaunchKernelGGL(k_reduce_partial, dim3(nblocks), dim3(256), 0, s, kind, N, W, c, K2, nv1, nbr1, v1, nv2,
                     nbr2, v2, nv3, nbr3, v3, partial, R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3((W + 255) / 256), dim3(256), 0, s, nblocks, W, partial, out);
  return hipGetLastError();
}

hipError_t launch_fibre_mass(hipStream_t s, int nf, const int32_t* ptr, const int32_t* rows, int W,
                             const double2* c, double* out) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fibre_mass, dim3(nf), dim3(256), 0, s, ptr, rows, W, c, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- allocation-free scratch
// Reduction partials of the allocation-free observables entry point live in this array, one
// copy per GPU for the life of the process.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): the address is looked up once
// per device with that device current and kept.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

hipError_t static_scratch(double** ptr) {
  static std::mutex mu;
  static double* per_device[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!per_device[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[dev] = static_cast<double*>(p);
  }
  *ptr = per_device[dev];
  return hipSuccess;
}

}  // namespace lsx

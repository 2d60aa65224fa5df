// Stochastic steps of liblsx: the semi-implicit step (Alg. 1) and its random batch form
// (Alg. 4) as one neighbour-stencil kernel, per-column fibre sampling (subsets without
// replacement, importance draws from a proposal), compaction of the sampled fibres' tiles,
// the per-fibre features and increment norms the proposal is trained on, and the proposal
// network itself (a width-64 tanh MLP in FP32: forward, backward, variance objective, Adam).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>

#include "lsx_internal.h"

namespace lsx {

// ---------------------------------------------------------------- semi-implicit / random batch
// out[i][w] = (x - i tau (a1 (V^1 x)_i + a2 (V^2 x)_i)) / (1 + i tau |K_i|^2 / 2), where
// (V^j x)_i = sum_p v_p x[nbr_j(i, p)] (the layer-j potential inside row i's fibre) and
// a_j = wt_j[fibre_j(i)][w] (1 when wt_j is null: Alg. 1).  One thread per (row, column).
//
// Cache blocking: every neighbour row is read again by nv other rows, the layer-1 ones
// (m - p, n) from far away in canonical order.  Workgroup b runs on XCD b % 8, so XCD x
// takes the contiguous slab x of the rows, and sweeps it in blocks of CW columns: the rows
// between a neighbour's first and last use then fit in that XCD's own L2.
//
// Stencil sizes NV1, NV2 are compile-time for the common cases (1D cosine: 2, 2D first shell:
// 6) so every neighbour index and value is loaded before any is used; a missing neighbour
// (index -1) reads a zero row instead of branching.  NV1 = 0 selects runtime loops.
template <int NVC>
__device__ __forceinline__ void si_stencil(int64_t i, int w, int W, int nv, const int32_t* __restrict__ nbr,
                                           const double2* __restrict__ v, const double2* __restrict__ X,
                                           const double2* __restrict__ zero, double& sr, double& si) {
  if (NVC > 0) {
    int j[8];
    double2 y[8];
#pragma unroll
    for (int p = 0; p < NVC; ++p) j[p] = nbr[i * NVC + p];
#pragma unroll
    for (int p = 0; p < NVC; ++p) y[p] = *(j[p] >= 0 ? X + (int64_t)j[p] * W + w : zero);
#pragma unroll
    for (int p = 0; p < NVC; ++p) {
      const double2 c = v[p];
      sr += c.x * y[p].x - c.y * y[p].y;
      si += c.x * y[p].y + c.y * y[p].x;
    }
  } else {
    for (int p = 0; p < nv; ++p) {
      const int jj = nbr[i * nv + p];
      const double2 y = *(jj >= 0 ? X + (int64_t)jj * W + w : zero), c = v[p];
      sr += c.x * y.x - c.y * y.y;
      si += c.x * y.y + c.y * y.x;
    }
  }
}

template <int NV1, int NV2>
__global__ __launch_bounds__(256) void k_si_step(int64_t N, int W, int CW, double tau, const double* __restrict__ K2,
                                                 int nv1, const int32_t* __restrict__ nbr1,
                                                 const double2* __restrict__ v1, const double* __restrict__ wt1,
                                                 const int32_t* __restrict__ fid1, int nv2,
                                                 const int32_t* __restrict__ nbr2, const double2* __restrict__ v2,
                                                 const double* __restrict__ wt2, const int32_t* __restrict__ fid2,
                                                 const double2* __restrict__ X, double2* __restrict__ Y,
                                                 const double2* __restrict__ zero) {
  const int xcd = blockIdx.x & 7;
  const int G = gridDim.x >> 3, lb = blockIdx.x >> 3;
  const int64_t slab = (N + 7) / 8;
  const int64_t r0 = xcd * slab, r1 = min(N, r0 + slab);
  const int rpi = 256 / CW;  // rows per workgroup iteration
  const int tr = threadIdx.x / CW, tc = threadIdx.x - tr * CW;
  for (int cb = 0; cb < W; cb += CW) {
    const int w = cb + tc;
    if (w >= W) continue;
    for (int64_t i = r0 + (int64_t)lb * rpi + tr; i < r1; i += (int64_t)G * rpi) {
      double s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
      si_stencil<NV1>(i, w, W, nv1, nbr1, v1, X, zero, s1r, s1i);
      si_stencil<NV2>(i, w, W, nv2, nbr2, v2, X, zero, s2r, s2i);
      const double a1 = wt1 ? wt1[(int64_t)fid1[i] * W + w] : 1.0;
      const double a2 = wt2 ? wt2[(int64_t)fid2[i] * W + w] : 1.0;
      const double2 x = X[i * W + w];
      // z = x - i tau (a1 s1 + a2 s2)
      const double zr = x.x + tau * (a1 * s1i + a2 * s2i);
      const double zi = x.y - tau * (a1 * s1r + a2 * s2r);
      // z / (1 + i b) = z (1 - i b) / (1 + b^2)
      const double b = 0.5 * tau * K2[i];
      const double den = 1.0 + b * b;
      Y[i * W + w] = make_double2((zr + b * zi) / den, (zi - b * zr) / den);
    }
  }
}

// ---------------------------------------------------------------- per-column sampling
// Random subset of p of the nf fibres for column w = blockIdx.x (Alg. 4): partial
// Fisher-Yates with the uniforms u[w][0..p-1] (position s swaps with
// s + floor(u (nf - s))), weight nf/p on the chosen fibres, 0 elsewhere; wt is [nf][W].
__global__ __launch_bounds__(256) void k_subset_weights(int nf, int W, int p, int ustride, const double* u,
                                                        double* wt) {
  extern __shared__ int32_t perm[];
  const int w = blockIdx.x;
  for (int f = threadIdx.x; f < nf; f += blockDim.x) perm[f] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double* uw = u + (int64_t)w * ustride;
    for (int s = 0; s < p; ++s) {
      int j = s + (int)floor(uw[s] * (double)(nf - s));
      j = j < nf - 1 ? j : nf - 1;
      const int tmp = perm[s];
      perm[s] = perm[j];
      perm[j] = tmp;
    }
  }
  __syncthreads();
  for (int f = threadIdx.x; f < nf; f += blockDim.x) wt[(int64_t)f * W + w] = 0.0;
  __syncthreads();
  const double g = (double)nf / (double)p;
  for (int s = threadIdx.x; s < p; s += blockDim.x) wt[(int64_t)perm[s] * W + w] = g;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Importance draws for column w = blockIdx.x: q = (1 - eps) softmax(z[w]) + eps / nf
// (uniform when z is null), cdf = running sum of q in fibre order, draw s lands on the
// first fibre whose cdf exceeds u[w][s] (the last fibre if none), and adds 1 / (p q_f)
// to that fibre's weight.  All draws of a fibre add the same value, so the sum does not
// depend on their order.  Dynamic LDS: 3 * nf doubles.  256 threads.
__global__ __launch_bounds__(256) void k_sample_weights(int nf, int W, int p, int ustride, const double* u,
                                                        const float* z, double eps, double* wt) {
  extern __shared__ double sm[];
  double* q = sm;
  double* cdf = sm + nf;
  double* acc = sm + 2 * nf;
  __shared__ double red[256];
  const int w = blockIdx.x;
  if (z) {
    const float* zw = z + (int64_t)w * nf;
    double mx = -INFINITY;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) mx = fmax(mx, (double)zw[f]);
    mx = block_max(mx, red);
    double s = 0.0;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      const double e = exp((double)zw[f] - mx);
      q[f] = e;
      s += e;
    }
    s = block_sum(s, red);
    for (int f = threadIdx.x; f < nf; f += blockDim.x) q[f] = (1.0 - eps) * q[f] / s + eps / nf;
  } else {
    for (int f = threadIdx.x; f < nf; f += blockDim.x) q[f] = 1.0 / nf;
  }
  for (int f = threadIdx.x; f < nf; f += blockDim.x) acc[f] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int f = 0; f < nf; ++f) {
      c += q[f];
      cdf[f] = c;
    }
  }
  __syncthreads();
  const double* uw = u + (int64_t)w * ustride;
  for (int s = threadIdx.x; s < p; s += blockDim.x) {
    const double us = uw[s];
    int lo = 0, hi = nf;  // first f with cdf[f] > us
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cdf[mid] > us)
        hi = mid;
      else
        lo = mid + 1;
    }
    const int f = lo < nf ? lo : nf - 1;
    atomicAdd(&acc[f], 1.0 / ((double)p * q[f]));
  }
  __syncthreads();
  for (int f = threadIdx.x; f < nf; f += blockDim.x) wt[(int64_t)f * W + w] = acc[f];
}

// Column list of every fibre: the columns (in increasing order) whose weight on it is
// nonzero.  One wave per fibre compacts 64 columns at a time with a ballot.
__global__ __launch_bounds__(256) void k_fibre_cols(int nf, int W, const double* wt, int32_t* cols, int32_t* ncols) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= nf) return;
  int base = 0;
  for (int w0 = 0; w0 < W; w0 += 64) {
    const int w = w0 + lane;
    const bool on = w < W && wt[(int64_t)f * W + w] != 0.0;
    const unsigned long long m = __ballot(on);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    if (on) cols[(int64_t)f * W + base + pos] = w;
    base += __popcll(m);
  }
  if (lane == 0) ncols[f] = base;
}

// Tile offsets of the sampled fibres: fibre f needs ceil(L_f / 16) row blocks times
// ceil(ncols_f / (16 NB)) column-slot blocks; off = exclusive scan in fibre order.
// One workgroup of 1024 threads; thread t scans fibres [t chunk, (t + 1) chunk).
__global__ __launch_bounds__(1024) void k_scan_tiles(int nf, int NB, const int32_t* ptr, const int32_t* ncols,
                                                     int32_t* off, int32_t* count) {
  __shared__ int32_t scan[1024];
  const int t = threadIdx.x;
  const int chunk = (nf + 1023) / 1024;
  const int f0 = min(nf, t * chunk), f1 = min(nf, f0 + chunk);
  const int cw = 16 * NB;
  int mine = 0;
  for (int f = f0; f < f1; ++f) mine += ((ptr[f + 1] - ptr[f] + 15) / 16) * ((ncols[f] + cw - 1) / cw);
  scan[t] = mine;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
    const int v = t >= o ? scan[t - o] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  int pos = scan[t] - mine;
  for (int f = f0; f < f1; ++f) {
    off[f] = pos;
    pos += ((ptr[f + 1] - ptr[f] + 15) / 16) * ((ncols[f] + cw - 1) / cw);
  }
  if (t == 1023) *count = scan[1023];
}

// Tiles of fibre f = blockIdx.x at off[f]: (row block rb, column-slot block cb), rb major, each with
// its row block's band when the band table is given (else the whole fibre).
__global__ __launch_bounds__(256) void k_emit_tiles(int NB, const int32_t* ptr, const int64_t* poff,
                                                    const int32_t* d0, const int32_t* bptr, const int32_t* band,
                                                    const int32_t* ncols, const int32_t* off, TileDesc* out) {
  const int f = blockIdx.x;
  const int r0 = ptr[f], L = ptr[f + 1] - r0;
  const int cw = 16 * NB;
  const int nc = (ncols[f] + cw - 1) / cw;
  const int n = ((L + 15) / 16) * nc;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    TileDesc t;
    t.r0 = r0;
    t.L = L;
    t.rb = k / nc;
    t.wb = k - t.rb * nc;
    t.poff = poff ? poff[f] : 0;
    t.f = f;
    t.d0 = d0 ? d0[f] : r0;
    t.k0 = band ? band[2 * (bptr[f] + t.rb)] : 0;
    t.k1 = band ? band[2 * (bptr[f] + t.rb) + 1] : kBandEnd;
    t.bb = -1;
    t.pad_ = 0;
    out[off[f] + k] = t;
  }
}

// Copies the (rows x gathered columns) block of every listed tile from src to dst (rows
// through pos when set); tiles at or past *count are skipped.  256 threads per tile.
__global__ __launch_bounds__(256) void k_copy_cols(const TileDesc* tiles, const int32_t* count, int NB,
                                                   const int32_t* pos, int W, const int32_t* cols,
                                                   const int32_t* ncols, const double2* src, double2* dst) {
  if ((int)blockIdx.x >= *count) return;
  const TileDesc t = tiles[blockIdx.x];
  const int rows = min(16, t.L - 16 * t.rb);
  const int cw = 16 * NB;
  const int s0 = t.wb * cw, ns = min(cw, ncols[t.f] - s0);
  for (int e = threadIdx.x; e < rows * cw; e += blockDim.x) {
    const int r = e / cw, c = e - r * cw;
    if (c >= ns) continue;
    const int w = cols[(int64_t)t.f * W + s0 + c];
    const int p = t.r0 + 16 * t.rb + r;
    const int64_t row = pos ? pos[p] : p;
    dst[row * W + w] = src[row * W + w];
  }
}

// ---------------------------------------------------------------- training data
// b[w][f] = sum over the fibre's rows of |Y - X|^2 (one workgroup per fibre)
__global__ __launch_bounds__(256) void k_fibre_incr(const int32_t* ptr, const int32_t* rows, int nf, int W,
                                                    const double2* X, const double2* Y, double* out) {
  __shared__ double red[256];
  const int f = blockIdx.x;
  const int r0 = ptr[f], L = ptr[f + 1] - r0;
  const int WB = W < 256 ? W : 256;
  const int S = 256 / WB;
  const int tid = threadIdx.x;
  for (int w0 = 0; w0 < W; w0 += WB) {
    const int w = w0 + tid % WB, s = tid / WB;
    double acc = 0.0;
    if (w < W && s < S)
      for (int a = s; a < L; a += S) {
        const int64_t e = (int64_t)rows[r0 + a] * W + w;
        const double dr = Y[e].x - X[e].x, di = Y[e].y - X[e].y;
        acc += dr * dr + di * di;
      }
    red[tid] = acc;
    __syncthreads();
    if (tid < WB && w0 + tid < W) {
      double sum = 0.0;
      for (int j = 0; j < S; ++j) sum += red[j * WB + tid];
      out[(int64_t)(w0 + tid) * nf + f] = sum;
    }
    __syncthreads();
  }
}

// X[w][f][:] = (shift / Kmax (d), |shift / Kmax|^2, log10(max(mass, 1e-30)) / 10, layer sign)
// from sfeat[f] = (shift / Kmax, |shift / Kmax|^2) and mass [nf][W].
__global__ __launch_bounds__(256) void k_features(int nf, int W, int d, const double* sfeat, const double* mass,
                                                  float sign, float* X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nf * W) return;
  const int w = (int)(e / nf), f = (int)(e - (int64_t)w * nf);
  const int nin = d + 3;
  float* x = X + e * nin;
  for (int k = 0; k <= d; ++k) x[k] = (float)sfeat[f * (d + 1) + k];
  x[d + 1] = (float)(log10(fmax(mass[(int64_t)f * W + w], 1e-30)) / 10.0);
  x[d + 2] = sign;
}

// ---------------------------------------------------------------- proposal network
// Flat FP32 parameters: W1 [nin][64], b1 [64], W2 [64][64], b2 [64], w3 [64], b3.
// z = w3 . tanh(W2^T tanh(W1^T x + b1) + b2) + b3.
constexpr int MLP_H = 64;
constexpr int MLP_NIN_MAX = 8;

struct MlpOff {
  int W1, b1, W2, b2, w3, b3, n;
  __host__ __device__ explicit MlpOff(int nin) {
    W1 = 0;
    b1 = nin * MLP_H;
    W2 = b1 + MLP_H;
    b2 = W2 + MLP_H * MLP_H;
    w3 = b2 + MLP_H;
    b3 = w3 + MLP_H;
    n = b3 + 1;
  }
};

int mlp_nparams(int nin) { return MlpOff(nin).n; }

__device__ __forceinline__ void mlp_stage(const float* theta, int n, float* sp) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) sp[k] = theta[k];
}

__device__ __forceinline__ void mlp_load_row(const float* X, int64_t M, int nin, int64_t m, float (&x)[MLP_NIN_MAX]) {
#pragma unroll
  for (int i = 0; i < MLP_NIN_MAX; ++i) x[i] = (m < M && i < nin) ? X[m * nin + i] : 0.f;
}

// The hidden-layer products are dense contractions over 64 units: H1 (rows x 64) W2, and in the
// backward pass D2 W2^T and H1^T D2.  Each wave takes chunks of 16 rows and forms them on the
// matrix cores with v_mfma_f32_16x16x4f32 (FP32 operands and accumulation, the network's own
// precision); the first layer (nin inputs), the tanh and the output layer stay on the VALU.
// Operand layouts of the instruction: A (16 x 4): lane l holds A[l % 16][l / 16]; B (4 x 16):
// lane l holds B[l / 16][l % 16]; C (16 x 16): element r of lane l is C[4 (l / 16) + r][l % 16].
typedef float mlp_v4f __attribute__((ext_vector_type(4)));
constexpr int MLP_CH = 16;    // rows per wave chunk
constexpr int MLP_LDT = 68;   // LDS row stride of a chunk's 64-wide tiles (floats)
constexpr int MLP_WTILE = 2 * MLP_CH * MLP_LDT + MLP_CH * MLP_NIN_MAX;  // per-wave LDS (H1, D, X)

// W2 in the B layout: w2[kk][ct] = W2[4 kk + lk][16 ct + li]
__device__ __forceinline__ void mlp_w2_frag(const float* sp, const MlpOff& o, int li, int lk, float (&w2)[16][4]) {
#pragma unroll
  for (int kk = 0; kk < 16; ++kk)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) w2[kk][ct] = sp[o.W2 + (4 * kk + lk) * MLP_H + 16 * ct + li];
}

// H1[li][4 kk + lk] for kk = 0..15 (the A layout of the layer-2 product), fed straight into it:
// acc[ct] = pre-activation of layer 2, rows 4 lk + r, units 16 ct + li.  H1 (may be null) gets
// the chunk's first-layer activations at [row][unit].  W2 operands from registers (w2, REG) or
// from the staged parameters in LDS.
template <bool REG>
__device__ __forceinline__ void mlp_hidden(const float* sp, const MlpOff& o, int nin, const float (&x)[MLP_NIN_MAX],
                                           int li, int lk, const float (*w2)[4], mlp_v4f (&acc)[4], float* H1) {
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = (mlp_v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int j = 4 * kk + lk;
    float a = sp[o.b1 + j];
#pragma unroll
    for (int i = 0; i < MLP_NIN_MAX; ++i)
      if (i < nin) a += x[i] * sp[o.W1 + i * MLP_H + j];
    const float h = tanhf(a);
    if (H1) H1[li * MLP_LDT + j] = h;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const float b = REG ? w2[kk][ct] : sp[o.W2 + (4 * kk + lk) * MLP_H + 16 * ct + li];
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(h, b, acc[ct], 0, 0, 0);
    }
  }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const float* theta, int nin, const float* X, int64_t M, float* z) {
  extern __shared__ float sp[];
  const MlpOff o(nin);
  mlp_stage(theta, o.n, sp);
  __syncthreads();
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4, wave = threadIdx.x >> 6;
  float w2[16][4], b2[4], w3[4];
  mlp_w2_frag(sp, o, li, lk, w2);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    b2[ct] = sp[o.b2 + 16 * ct + li];
    w3[ct] = sp[o.w3 + 16 * ct + li];
  }
  const float b3 = sp[o.b3];
  const int64_t nch = (M + MLP_CH - 1) / MLP_CH;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < nch; c += (int64_t)gridDim.x * 4) {
    float x[MLP_NIN_MAX];
    mlp_load_row(X, M, nin, c * MLP_CH + li, x);
    mlp_v4f acc[4];
    mlp_hidden<true>(sp, o, nin, x, li, lk, w2, acc, nullptr);
    float zr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      zr[r] = 0.f;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) zr[r] += tanhf(acc[ct][r] + b2[ct]) * w3[ct];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) zr[r] += __shfl_xor(zr[r], off);
    }
    if (li == 0)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = c * MLP_CH + 4 * lk + r;
        if (m < M) z[m] = zr[r] + b3;
      }
  }
}

// Backward of sum_m g_m z_m, g_m = dz[m] * (*gscale when set):
//   d2 = g w3 (1 - h2^2),  d1 = (d2 W2^T)(1 - h1^2),
//   grad W2 = H1^T d2 (matrix cores, accumulated in registers over the wave's chunks),
//   grad W1 = X^T d1, b1, b2, w3, b3: sums over rows.
// Each wave stages its chunk's H1, d2 (then d1) and inputs in its own LDS tiles; the waves'
// sums are added in wave order at the end and the workgroup writes partial[blockIdx.x][:].
__global__ __launch_bounds__(256) void k_mlp_bwd(const float* theta, int nin, const float* X, int64_t M,
                                                 const float* dz, const double* gscale, float* partial) {
  extern __shared__ float sp[];
  const MlpOff o(nin);
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4, wave = threadIdx.x >> 6;
  float* H1 = sp + ((o.n + 3) & ~3) + wave * MLP_WTILE;
  float* D = H1 + MLP_CH * MLP_LDT;
  float* XS = D + MLP_CH * MLP_LDT;
  mlp_stage(theta, o.n, sp);
  __syncthreads();
  const float gs = gscale ? (float)*gscale : 1.f;
  float b2[4], w3[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    b2[ct] = sp[o.b2 + 16 * ct + li];
    w3[ct] = sp[o.w3 + 16 * ct + li];
  }
  mlp_v4f gW2[4][4];  // [jt][kt]: grad W2[16 jt + 4 lk + r][16 kt + li]
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) gW2[jt][kt] = (mlp_v4f){0.f, 0.f, 0.f, 0.f};
  float gb2[4] = {0.f, 0.f, 0.f, 0.f}, gw3[4] = {0.f, 0.f, 0.f, 0.f};  // units 16 ct + li, rows 4 lk + r
  float gW1[MLP_NIN_MAX], gb1 = 0.f, gb3 = 0.f;                          // unit = lane
#pragma unroll
  for (int i = 0; i < MLP_NIN_MAX; ++i) gW1[i] = 0.f;
  const int64_t nch = (M + MLP_CH - 1) / MLP_CH;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < nch; c += (int64_t)gridDim.x * 4) {
    float x[MLP_NIN_MAX];
    mlp_load_row(X, M, nin, c * MLP_CH + li, x);
    if (lk == 0)
#pragma unroll
      for (int i = 0; i < MLP_NIN_MAX; ++i) XS[li * MLP_NIN_MAX + i] = x[i];
    mlp_v4f acc[4];
    mlp_hidden<false>(sp, o, nin, x, li, lk, nullptr, acc, H1);
    float g[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = c * MLP_CH + 4 * lk + r;
      g[r] = (m < M) ? dz[m] * gs : 0.f;
    }
    if (li == 0) gb3 += (g[0] + g[1]) + (g[2] + g[3]);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float h2 = tanhf(acc[ct][r] + b2[ct]);
        const float d2 = g[r] * w3[ct] * (1.f - h2 * h2);
        D[(4 * lk + r) * MLP_LDT + 16 * ct + li] = d2;
        gb2[ct] += d2;
        gw3[ct] += g[r] * h2;
      }
    // the chunk's tiles are written by other lanes of this wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // grad W2 += H1^T d2 (k-steps over the chunk's rows)
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int row = 4 * s4 + lk;
      float a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = H1[row * MLP_LDT + 16 * t + li];
        b[t] = D[row * MLP_LDT + 16 * t + li];
      }
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
          gW2[jt][kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[jt], b[kt], gW2[jt][kt], 0, 0, 0);
    }
    // e = d2 W2^T: rows 4 lk + r, units 16 jt + li
    mlp_v4f e[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) e[jt] = (mlp_v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const float a = D[li * MLP_LDT + 4 * kk + lk];
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
        e[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, sp[o.W2 + (16 * jt + li) * MLP_H + 4 * kk + lk], e[jt], 0,
                                                     0, 0);
    }
    // d1 = e (1 - h1^2), written over d2 (every lane has read its d2 operands above)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * lk + r, j = 16 * jt + li;
        const float h = H1[row * MLP_LDT + j];
        D[row * MLP_LDT + j] = e[jt][r] * (1.f - h * h);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // grad W1, b1 for unit j = lane over the chunk's rows
#pragma unroll 4
    for (int row = 0; row < MLP_CH; ++row) {
      const float d1 = D[row * MLP_LDT + lane];
      gb1 += d1;
#pragma unroll
      for (int i = 0; i < MLP_NIN_MAX; ++i) gW1[i] += XS[row * MLP_NIN_MAX + i] * d1;
    }
    // the tiles are rewritten by the next chunk
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // sums over the lane groups lk (rows) of the unit-per-lane-group terms
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    gb2[ct] += __shfl_xor(gb2[ct], 16);
    gb2[ct] += __shfl_xor(gb2[ct], 32);
    gw3[ct] += __shfl_xor(gw3[ct], 16);
    gw3[ct] += __shfl_xor(gw3[ct], 32);
  }
  gb3 += __shfl_xor(gb3, 16);
  gb3 += __shfl_xor(gb3, 32);
  // the waves' sums, added in wave order into sp (theta is no longer needed)
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
      auto put = [&](int idx, float v) { sp[idx] = (w == 0) ? v : sp[idx] + v; };
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) put(o.W2 + (16 * jt + 4 * lk + r) * MLP_H + 16 * kt + li, gW2[jt][kt][r]);
      for (int i = 0; i < nin; ++i) put(o.W1 + i * MLP_H + lane, gW1[i]);
      put(o.b1 + lane, gb1);
      if (lk == 0)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          put(o.b2 + 16 * ct + li, gb2[ct]);
          put(o.w3 + 16 * ct + li, gw3[ct]);
        }
      if (lane == 0) put(o.b3, gb3);
    }
    __syncthreads();
  }
  float* out = partial + (int64_t)blockIdx.x * o.n;
  for (int k = threadIdx.x; k < o.n; k += blockDim.x) out[k] = sp[k];
}

// grad[e] = sum over workgroups of partial[b][e] (FP64, fixed order)
__global__ __launch_bounds__(256) void k_mlp_reduce(int nparts, int n, const float* partial, float* grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += partial[(int64_t)b * n + e];
  grad[e] = (float)s;
}

// Variance objective per group g (rows gptr[g]..gptr[g+1]), one workgroup per group:
// q = (1 - eps) softmax(z) + eps / n, l_g = sum b/q / (sum sqrt b)^2 and the unscaled
// gradient (1 - eps)/S sigma_f (sum_h r_h sigma_h - r_f), r = b / q^2; groups with
// sum b = 0 get l_g = 0, active = 0 and zero gradient.
__global__ __launch_bounds__(256) void k_loss_groups(const float* z, const double* b, const int64_t* gptr,
                                                     int64_t G, double eps, double* lg, int32_t* active,
                                                     float* dz) {
  __shared__ double red[256];
  for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
    const int64_t r0 = gptr[g], r1 = gptr[g + 1];
    const double n = (double)(r1 - r0);
    double mx = -INFINITY, sb = 0.0, ss = 0.0;
    for (int64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) {
      mx = fmax(mx, (double)z[k]);
      sb += b[k];
      ss += sqrt(b[k]);
    }
    mx = block_max(mx, red);
    sb = block_sum(sb, red);
    ss = block_sum(ss, red);
    if (!(sb > 0.0)) {
      for (int64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) dz[k] = 0.f;
      if (threadIdx.x == 0) {
        lg[g] = 0.0;
        active[g] = 0;
      }
      continue;
    }
    double se = 0.0;
    for (int64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) se += exp((double)z[k] - mx);
    se = block_sum(se, red);
    double sl = 0.0, srs = 0.0;
    for (int64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) {
      const double sig = exp((double)z[k] - mx) / se;
      const double qf = (1.0 - eps) * sig + eps / n;
      sl += b[k] / qf;
      srs += b[k] / (qf * qf) * sig;
    }
    sl = block_sum(sl, red);
    srs = block_sum(srs, red);
    const double S = ss * ss;
    for (int64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) {
      const double sig = exp((double)z[k] - mx) / se;
      const double qf = (1.0 - eps) * sig + eps / n;
      const double rf = b[k] / (qf * qf);
      dz[k] = (float)((1.0 - eps) / S * sig * (srs - rf));
    }
    if (threadIdx.x == 0) {
      lg[g] = sl / S;
      active[g] = 1;
    }
  }
}

// out[0] = mean of l_g over active groups, out[1] = 1 / (number of active groups) (0 if none)
__global__ __launch_bounds__(256) void k_loss_final(int64_t G, const double* lg, const int32_t* active,
                                                    double* out) {
  __shared__ double red[256];
  double s = 0.0, a = 0.0;
  for (int64_t g = threadIdx.x; g < G; g += blockDim.x) {
    s += lg[g];
    a += active[g];
  }
  s = block_sum(s, red);
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    out[0] = a > 0.0 ? s / a : 0.0;
    out[1] = a > 0.0 ? 1.0 / a : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_scale_f32(int64_t n, const double* scale, float* x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = (float)((double)x[e] * *scale);
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// theta -= lr (m c1) / (sqrt(v c2) + eps) with c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ __launch_bounds__(256) void k_adam(int n, float* theta, float* m, float* v, const float* grad,
                                              double lr, double b1, double b2, double eps, double c1, double c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double g = grad[e];
  const double mm = b1 * m[e] + (1.0 - b1) * g;
  const double vv = b2 * v[e] + (1.0 - b2) * g * g;
  m[e] = (float)mm;
  v[e] = (float)vv;
  theta[e] = (float)((double)theta[e] - lr * (mm * c1) / (sqrt(vv * c2) + eps));
}

// ================================================================ launchers
static unsigned grid_for(int64_t n, int64_t cap) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_si_step(hipStream_t s, int64_t N, int W, double tau, const double* K2, int nv1,
                          const int32_t* nbr1, const double2* v1, const double* wt1, const int32_t* fid1, int nv2,
                          const int32_t* nbr2, const double2* v2, const double* wt2, const int32_t* fid2,
                          const double2* X, double2* Y, const double2* zero) {
  if (N == 0) return hipSuccess;
  // column block: LSX_SI_CW (1..256, a power of two) or 8; 256 workgroups per XCD
  static const int cw_env = [] {
    const char* v = std::getenv("LSX_SI_CW");
    const int x = v ? std::atoi(v) : 8;
    return (x >= 1 && x <= 256 && (x & (x - 1)) == 0) ? x : 8;
  }();
  int CW = cw_env;
  while (CW > 1 && CW / 2 >= W) CW /= 2;  // narrow states: no idle lanes beyond W
  const int64_t rows_per_xcd = (N + 7) / 8;
  const int64_t G = std::min<int64_t>(256, std::max<int64_t>(1, (rows_per_xcd * CW + 255) / 256));
  const dim3 grid((unsigned)(8 * G));
  if (nv1 == 2 && nv2 == 2)
    hipLaunchKernelGGL((k_si_step<2, 2>), grid, dim3(256), 0, s, N, W, CW, tau, K2, nv1, nbr1, v1, wt1, fid1, nv2,
                       nbr2, v2, wt2, fid2, X, Y, zero);
  else if (nv1 == 6 && nv2 == 6)
    hipLaunchKernelGGL((k_si_step<6, 6>), grid, dim3(256), 0, s, N, W, CW, tau, K2, nv1, nbr1, v1, wt1, fid1, nv2,
                       nbr2, v2, wt2, fid2, X, Y, zero);
  else
    hipLaunchKernelGGL((k_si_step<0, 0>), grid, dim3(256), 0, s, N, W, CW, tau, K2, nv1, nbr1, v1, wt1, fid1, nv2,
                       nbr2, v2, wt2, fid2, X, Y, zero);
  return hipGetLastError();
}

hipError_t launch_subset_weights(hipStream_t s, int nf, int W, int p, int ustride, const double* u, double* wt) {
  hipLaunchKernelGGL(k_subset_weights, dim3(W), dim3(256), (size_t)nf * sizeof(int32_t), s, nf, W, p, ustride, u,
                     wt);
  return hipGetLastError();
}

hipError_t launch_sample_weights(hipStream_t s, int nf, int W, int p, int ustride, const double* u, const float* z,
                                 double eps, double* wt) {
  hipLaunchKernelGGL(k_sample_weights, dim3(W), dim3(256), (size_t)3 * nf * sizeof(double), s, nf, W, p, ustride,
                     u, z, eps, wt);
  return hipGetLastError();
}

hipError_t launch_sampled_tiles(hipStream_t s, int nf, int W, int NB, const double* wt, const int32_t* ptr,
                                const int64_t* poff, const int32_t* d0, const int32_t* bptr, const int32_t* band,
                                int32_t* cols, int32_t* ncols, int32_t* off, TileDesc* tiles, int32_t* count) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fibre_cols, dim3((nf + 3) / 4), dim3(256), 0, s, nf, W, wt, cols, ncols);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, nf, NB, ptr, ncols, off, count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_emit_tiles, dim3(nf), dim3(256), 0, s, NB, ptr, poff, d0, bptr, band, ncols, off, tiles);
  return hipGetLastError();
}

hipError_t launch_copy_cols(hipStream_t s, int ntiles, const TileDesc* tiles, const int32_t* count, int NB,
                            const int32_t* pos, int W, const int32_t* cols, const int32_t* ncols, const double2* src,
                            double2* dst) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, dim3(ntiles), dim3(256), 0, s, tiles, count, NB, pos, W, cols, ncols, src, dst);
  return hipGetLastError();
}

hipError_t launch_fibre_incr(hipStream_t s, int nf, const int32_t* ptr, const int32_t* rows, int W,
                             const double2* X, const double2* Y, double* out) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fibre_incr, dim3(nf), dim3(256), 0, s, ptr, rows, nf, W, X, Y, out);
  return hipGetLastError();
}

hipError_t launch_features(hipStream_t s, int nf, int W, int d, const double* sfeat, const double* mass,
                           float sign, float* X) {
  const int64_t n = (int64_t)nf * W;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nf, W, d, sfeat, mass, sign,
                     X);
  return hipGetLastError();
}

static size_t mlp_lds_fwd(int nin) { return (size_t)((MlpOff(nin).n + 3) & ~3) * sizeof(float); }
static size_t mlp_lds_bwd(int nin) {
  return (size_t)(((MlpOff(nin).n + 3) & ~3) + 4 * MLP_WTILE) * sizeof(float);
}

// workgroups of the backward pass (4 waves of 16-row chunks each): one partial gradient each
int mlp_bwd_blocks(int64_t M) {
  const int64_t nblk = (M + 4 * MLP_CH - 1) / (4 * MLP_CH);
  return (int)(nblk < 1 ? 1 : (nblk > 512 ? 512 : nblk));
}

hipError_t launch_mlp_fwd(hipStream_t s, const float* theta, int nin, const float* X, int64_t M, float* z) {
  if (M == 0) return hipSuccess;
  const int64_t nblk = (M + 4 * MLP_CH - 1) / (4 * MLP_CH);
  const unsigned grid = (unsigned)(nblk > 2048 ? 2048 : nblk);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(grid), dim3(256), mlp_lds_fwd(nin), s, theta, nin, X, M, z);
  return hipGetLastError();
}

hipError_t launch_mlp_bwd(hipStream_t s, const float* theta, int nin, const float* X, int64_t M, const float* dz,
                          const double* gscale, float* partial, float* grad) {
  const int nparts = mlp_bwd_blocks(M);
  const int n = MlpOff(nin).n;
  hipLaunchKernelGGL(k_mlp_bwd, dim3(nparts), dim3(256), mlp_lds_bwd(nin), s, theta, nin, X, M, dz, gscale, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((n + 255) / 256), dim3(256), 0, s, nparts, n, partial, grad);
  return hipGetLastError();
}

hipError_t launch_loss(hipStream_t s, const float* z, const double* b, const int64_t* gptr, int64_t G, double eps,
                       double* lg, int32_t* active, float* dz, double* out) {
  if (G == 0) return hipSuccess;
  const unsigned grid = (unsigned)(G > 65536 ? 65536 : G);
  hipLaunchKernelGGL(k_loss_groups, dim3(grid), dim3(256), 0, s, z, b, gptr, G, eps, lg, active, dz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, G, lg, active, out);
  return hipGetLastError();
}

hipError_t launch_scale_f32(hipStream_t s, int64_t n, const double* scale, float* x) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, scale, x);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, int n, float* theta, float* m, float* v, const float* grad, double lr,
                       double b1, double b2, double eps, double c1, double c2) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, n, theta, m, v, grad, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lsx

// Internal declarations shared by the host library and the HIP kernels of liblsx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lsx.h"

namespace lsx {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
#define LSX_HIP_TRY(expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      ::lsx::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                  \
      return LSX_E_HIP;                                                                     \
    }                                                                                       \
  } while (0)

// ---------------------------------------------------------------- storage formats
// Propagator storage, per fibre f of length L (all formats zero-padded):
//  PF_F64    : complex128 P, Lp = roundup(L,16); chunk (rb, ks) = rows 16rb.., cols 4ks..
//              holds 64 double2, lane l = (row%16) + 16*(col%4).  Chunk index rb*(Lp/4)+ks.
//              This is exactly the A-operand order of v_mfma_f64_16x16x4f64.
//  PF_F32    : the off-diagonal part E of P as complex64 in the same chunk order
//              (A-operand order of v_mfma_f32_16x16x4f32), diagonal held in FP64 separately.
//  PF_BF16X3 : E split into three bf16 terms; Lp = roundup(L,32); chunk (rb, kc) = rows
//              16rb.., cols 32kc..; per chunk 6 planes (term*2 + {re,im}) of 64 lanes x 8
//              bf16, lane l = (row%16) + 16*((col%32)/8), element col%8 -- the A-operand
//              order of v_mfma_f32_16x16x32_bf16.
enum PropFormat { PF_F64 = 0, PF_F32 = 1, PF_BF16X3 = 2 };

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
inline int prop_pad(int fmt) { return fmt == PF_BF16X3 ? 32 : 16; }
// size in bytes of one fibre's propagator storage
inline int64_t prop_bytes(int fmt, int L) {
  int64_t Lp = round_up(L, prop_pad(fmt));
  switch (fmt) {
    case PF_F64: return Lp * Lp * 16;
    case PF_F32: return Lp * Lp * 8;
    default: return Lp * Lp * 12;  // 3 terms x (re, im) x bf16
  }
}

// Tile of a fibre pass (48 bytes, read with scalar loads): fibre f starting at fibre
// position r0 with length L, output rows 16*rb.., columns 16*NB*wb.., the byte offset of
// the fibre's propagator and of its diagonal, and the band [k0, k1) of fibre positions
// whose propagator columns hold an entry above the plan's band tolerance for any of the
// tile's rows (multiples of the format's column chunk; the kernels clamp k1 to the padded
// fibre length, so k1 = INT32_MAX means "to the end").  bb: entry of the propagator's first
// 16-row block in the per-block band table (PassArgs::rb_band), -1 when the tile has none.
// f < 0 marks a padding tile.
struct TileDesc {
  int32_t r0, L, rb, wb;
  int64_t poff;
  int32_t f;
  int32_t d0;  // mixed formats: position of this propagator's diagonal (fibres may share one)
  int32_t k0, k1;
  int32_t bb, pad_;
};
constexpr int32_t kBandEnd = 0x7fffffff;
// columns per propagator chunk of a format (the unit of the band)
inline int band_chunk(int fmt) { return fmt == PF_BF16X3 ? 32 : 4; }
// Fibres sharing a stored propagator are grouped by up to kOrbitMax; single-state passes
// over such groups use the tile shape nb = kOrbitNB (PassArgs::orbit).
constexpr int kOrbitMax = 8;
constexpr int kOrbitStride = 1 + kOrbitMax;
constexpr int kOrbitNB = 8;

struct PassArgs;
// Arguments of every fibre-pass kernel.  Element k of fibre f (fibre position
// p = r0 + k) is row in_pos[p] of X and row out_pos[p] of Y (identity when null),
// so a pass can read one array layout and write another.
// Weighted passes (wt set): the output is x + wt[f][w] (P_f x - x) per fibre f and column
// w, i.e. a weighted fibre increment; tcount (device) bounds the tiles a launch runs.
struct PassArgs {
  const TileDesc* tiles = nullptr;
  const int32_t* in_pos = nullptr;
  const int32_t* out_pos = nullptr;
  const int32_t* ph_idx = nullptr;  // canonical index of fibre position p (identity when null)
  const double2* ph = nullptr;      // kinetic phase applied to the output rows (none when null)
  const void* P = nullptr;          // propagator storage (format per kernel)
  const double2* diag = nullptr;    // mixed formats: diagonal of P at fibre position p
  const double2* X = nullptr;       // input state  [rows][W]
  double2* Y = nullptr;             // output state [rows][W]
  const void* zero = nullptr;       // >= 256 zero bytes: target of every out-of-range operand load
  const PassArgs* batch = nullptr;  // batched launches: per-system arguments, indexed by TileDesc::f
  const double* wt = nullptr;       // weighted passes: [fibre][W] increment weights
  const int32_t* tcount = nullptr;  // device tile count: workgroups at or past it exit
  // column-gathered passes: column slot s of fibre f is state column cols[f][s] for
  // s < ncols[f] (TileDesc::wb then counts blocks of 16 NB slots, not of columns)
  const int32_t* cols = nullptr;
  const int32_t* ncols = nullptr;
  // row-split passes: band of every 16-row block of the layer's stored propagators, (k0, k1)
  // fibre positions at [2 (TileDesc::bb + block)]; each wave of a tile then skips the chunks
  // outside its own block's band (null: the tile's band for every wave)
  const int32_t* rb_band = nullptr;
  // persistent batched launches: mode (0 none, 1 per-XCD tile queues on device counters,
  // 2 static stride), 9 device counters that are zero between launches (mode 1) and the
  // number of tiles in `tiles`
  int32_t persist = 0;
  int32_t* queue = nullptr;
  int32_t ntiles = 0;
  int32_t W = 0;
  // output stores: 0 ordinary (lines kept in the writer's L2), 1 non-temporal (streamed out);
  // the faster one depends on the state's size and is measured per state
  int32_t nt = 0;
  // K-split FP64 / FP32 passes: groups of k-steps each wave keeps in flight (1, 2 or 4; 0: the
  // library default), chosen per state by the tile tuner
  int32_t u = 0;
  // single-state orbit passes (W = 1, tile shape nb = kOrbitNB): TileDesc::f indexes this
  // table of fibre groups that share one stored propagator, kOrbitStride entries per group:
  // the member count, then the fibre position of every member's first row (entries past the
  // count repeat the first member's); orbit_max is the largest group of the layer
  const int32_t* orbit = nullptr;
  int32_t orbit_max = 0;
};

// ---------------------------------------------------------------- kernel launchers (lsx_kernels.hip)
hipError_t launch_assemble(hipStream_t s, int nb, const int32_t* fid, const int32_t* ptr, const int32_t* rows,
                           const int32_t* mn, int d, int stride, int own, double kfac, const double* K2, int nv,
                           const int32_t* vidx, const double* vre, const double* vim, int embed, double* A,
                           const int64_t* moff, const int32_t* ndim);
// Blocked two-sided Jacobi (long fibres): arguments of one round.  Matrices are indexed by their
// slot m (moff, ndim: padded size, a multiple of 32).  mat lists this sweep's unconverged
// matrices by size, largest first; a round runs on the first `count` of them (those with more
// than `round` + 1 blocks of 16).  pfx_pairs / pfx_tiles are prefix sums over mat of nb/2 pairs
// and 2 (nb/2)^2 tiles (nb = n/16); Q holds every pair's 32x32 rotation (row-major) at its
// pfx_pairs index; flag[m] is set to 1 when matrix m was rotated; tiny[m] is its skip threshold.
struct BJArgs {
  double* A = nullptr;
  double* VT = nullptr;
  const int64_t* moff = nullptr;
  const int32_t* ndim = nullptr;
  double* tiny = nullptr;
  const int32_t* mat = nullptr;
  const int32_t* pfx_pairs = nullptr;
  const int32_t* pfx_tiles = nullptr;
  int count = 0;
  int round = 0;
  double* Q = nullptr;
  int32_t* flag = nullptr;
};
hipError_t launch_bj_init(hipStream_t s, int nsel, const int32_t* sel, const BJArgs& g);
hipError_t launch_bj_round(hipStream_t s, int npairs, int ntiles, const BJArgs& g);
hipError_t launch_bj_finish(hipStream_t s, int nsel, const int32_t* sel, const BJArgs& g, double* lam,
                            const int64_t* loff);

// Scalar cyclic Jacobi, one workgroup per matrix; sel (nullable) lists the matrices to solve.
hipError_t launch_jacobi(hipStream_t s, int nf, int maxn, double* A, double* VT, const int64_t* moff,
                         const int32_t* ndim, double* lam, const int64_t* loff, int32_t* info,
                         int maxsweeps, const int32_t* sel = nullptr);
hipError_t launch_eig_fn(hipStream_t s, int64_t nlam, const double* lam, double t, int flow, double2* gh);
hipError_t launch_form(hipStream_t s, int fmt, int nb, int maxL, const int32_t* fid, const int32_t* ptr,
                       const double* VT, const int64_t* moff, const int32_t* ndim, const int32_t* embed,
                       const double2* gh, const int64_t* loff, void* P, const int64_t* poff, double2* diag);
// Band of every 16-row block of every stored propagator (k_band): band[2 (boff[b] + rb)] and
// band[2 (boff[b] + rb) + 1] = first and one past the last column chunk with an entry whose
// |Re| + |Im| >= tol (a block with none keeps its diagonal chunk).
hipError_t launch_band(hipStream_t s, int fmt, int nb, const int32_t* fid, const int32_t* ptr, const void* P,
                       const int64_t* poff, const int64_t* boff, double tol, int32_t* band);
hipError_t launch_phase_table(hipStream_t s, int64_t N, const double* K2, double theta_scale, double2* ph);
hipError_t launch_phase_apply(hipStream_t s, int64_t N, int W, const double2* ph, double2* c);
hipError_t launch_pass(hipStream_t s, int fmt, int W, int ntiles, int nb, int ksplit, const PassArgs& a,
                       bool batched = false);
// Batched launches with a.persist set: computes (once per kernel) the persistent grid of the pass
// kernel launch_pass would use, launching nothing, so no occupancy query runs under capture.
hipError_t prepare_persistent(int fmt, int W, int nb, int ksplit, const PassArgs& a);
hipError_t launch_reduce(hipStream_t s, int kind, int64_t N, int W, const double2* c, const double* K2, int nv1,
                         const int32_t* nbr1, const double2* v1, int nv2, const int32_t* nbr2, const double2* v2,
                         int nv3, const int32_t* nbr3, const double2* v3, double* partial, int nblocks,
                         double* out);
hipError_t launch_fibre_mass(hipStream_t s, int nf, const int32_t* ptr, const int32_t* rows, int W,
                             const double2* c, double* out);
// Device address of this GPU's static scratch array (kStaticScratchDoubles doubles), looked up
// once per device on first use; never allocates.
constexpr int64_t kStaticScratchDoubles = int64_t(1) << 20;  // 8 MiB per GPU
constexpr int kMaxDevices = 64;
hipError_t static_scratch(double** ptr);

// ---------------------------------------------------------------- stochastic steps (lsx_sample.hip)
hipError_t launch_si_step(hipStream_t s, int64_t N, int W, double tau, const double* K2, int nv1,
                          const int32_t* nbr1, const double2* v1, const double* wt1, const int32_t* fid1, int nv2,
                          const int32_t* nbr2, const double2* v2, const double* wt2, const int32_t* fid2,
                          const double2* X, double2* Y, const double2* zero);
hipError_t launch_subset_weights(hipStream_t s, int nf, int W, int p, int ustride, const double* u, double* wt);
hipError_t launch_sample_weights(hipStream_t s, int nf, int W, int p, int ustride, const double* u, const float* z,
                                 double eps, double* wt);
// column lists of the sampled fibres and their tiles (16 NB column slots per tile)
// bptr, band (nullable): band of fibre f's row block rb at band[2 (bptr[f] + rb)] (k0, then k1)
hipError_t launch_sampled_tiles(hipStream_t s, int nf, int W, int NB, const double* wt, const int32_t* ptr,
                                const int64_t* poff, const int32_t* d0, const int32_t* bptr, const int32_t* band,
                                int32_t* cols, int32_t* ncols, int32_t* off, TileDesc* tiles, int32_t* count);
hipError_t launch_copy_cols(hipStream_t s, int ntiles, const TileDesc* tiles, const int32_t* count, int NB,
                            const int32_t* pos, int W, const int32_t* cols, const int32_t* ncols, const double2* src,
                            double2* dst);
hipError_t launch_fibre_incr(hipStream_t s, int nf, const int32_t* ptr, const int32_t* rows, int W,
                             const double2* X, const double2* Y, double* out);
hipError_t launch_features(hipStream_t s, int nf, int W, int d, const double* sfeat, const double* mass,
                           float sign, float* X);
// proposal network (width 64, FP32)
int mlp_nparams(int nin);
int mlp_bwd_blocks(int64_t M);
hipError_t launch_mlp_fwd(hipStream_t s, const float* theta, int nin, const float* X, int64_t M, float* z);
hipError_t launch_mlp_bwd(hipStream_t s, const float* theta, int nin, const float* X, int64_t M, const float* dz,
                          const double* gscale, float* partial, float* grad);
hipError_t launch_loss(hipStream_t s, const float* z, const double* b, const int64_t* gptr, int64_t G, double eps,
                       double* lg, int32_t* active, float* dz, double* out);
hipError_t launch_scale_f32(hipStream_t s, int64_t n, const double* scale, float* x);
hipError_t launch_adam(hipStream_t s, int n, float* theta, float* m, float* v, const float* grad, double lr,
                       double b1, double b2, double eps, double c1, double c2);

}  // namespace lsx

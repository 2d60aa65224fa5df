/*
 * lsx.h -- C-ABI of the MI355X layer-splitting library (liblsx.so).
 *
 * Computes the exact-flow layer-splitting time stepping of Wang, Chen, Zhou &
 * Zhou, "Layer-splitting methods for time-dependent Schroedinger equations of
 * incommensurate systems" (arXiv 2103.14897), on the lifted plane-wave
 * coefficient array phi_mn (Sec. 3, eqs. 3.2-3.6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns lsx_status: LSX_OK (0) or a negative error code.
 *    On error a thread-local message is available from lsx_last_error() and no
 *    output argument is written; handles are left unchanged.
 *  - Validation happens on the host before anything is enqueued.
 *  - Host arrays passed in are owned by the caller and are copied (or fully
 *    consumed) before the call returns, except where a stream-ordered upload is
 *    documented: then the caller keeps the buffer alive until the stream has
 *    reached that point.
 *  - Handles (lsx_system, lsx_plan, lsx_state) are owned by the library and
 *    freed by the matching *_destroy call.  A system must outlive its plans and
 *    a plan its states (destroying a parent with live children returns
 *    LSX_E_STATE and destroys nothing).
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.  All
 *    device work of a call is enqueued on that stream, in order.
 *  - Complex numbers are stored interleaved (re, im) as pairs of doubles.
 *  - A state holds W wavepackets as a device array c[N][W] of complex doubles
 *    (W innermost): c[i*W + w] is the coefficient of lifted index i (canonical
 *    order, see lsx_index_get) in wavepacket w.
 */
#ifndef LSX_H
#define LSX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSX_OK = 0,
  LSX_E_INVALID = -1,       /* bad argument (size, enum, pointer, geometry) */
  LSX_E_NOT_HERMITIAN = -2, /* potential coefficients violate v_{-m} = conj(v_m) */
  LSX_E_OOM = -3,           /* host or device allocation failed */
  LSX_E_HIP = -4,           /* a HIP runtime call failed; message has the HIP string */
  LSX_E_EIG = -5,           /* fibre eigensolver did not converge */
  LSX_E_NONFINITE = -6,     /* an observable came out NaN or Inf */
  LSX_E_STATE = -7          /* handle misuse (live children, mismatched plan, ...) */
} lsx_status;

enum { LSX_CUTOFF_BALL = 0, LSX_CUTOFF_PRODUCT = 1 };
enum {
  LSX_LIE = 0,       /* exact fibre flows, Lie order F1 F2 (App. A)                       */
  LSX_STRANG = 1,    /* exact fibre flows, Strang F1(tau/2) F2(tau) F1(tau/2) (App. A)    */
  LSX_LIE_BE = 2,    /* backward Euler fibre solves, Lie order (Alg. 2, eqs. 4.3-4.4)      */
  LSX_STRANG_CN = 3, /* Crank-Nicolson fibre solves, Strang order (eq. 4.6)              */
  LSX_YOSHIDA4 = 4   /* exact flows, fourth order: Strang steps of g1 tau, g0 tau, g1 tau  */
};
enum { LSX_FP64 = 0, LSX_MIX_FP32 = 1, LSX_MIX_BF16X3 = 2 };
enum {
  LSX_OBS_MASS = 1,         /* W doubles */
  LSX_OBS_ENERGY = 2,       /* W doubles */
  LSX_OBS_FIBRE_MASS_1 = 4, /* nfibres_1 * W doubles, [fibre][w] */
  LSX_OBS_FIBRE_MASS_2 = 8, /* nfibres_2 * W doubles, [fibre][w] */
  LSX_OBS_FIBRE_MASS_3 = 16 /* nfibres_3 * W doubles, [fibre][w] (three-layer systems) */
};

typedef struct lsx_system lsx_system;
typedef struct lsx_plan lsx_plan;
typedef struct lsx_state lsx_state;

/* Message of the last failed call on this thread ("" if none).  Never NULL. */
const char* lsx_last_error(void);

/*
 * Diagnostics: device buffers the library holds right now (every system, plan, state, batch,
 * sampler and network together) and their bytes.  After a failed call the counts are those
 * before it: set-up failures unwind what they allocated.  Either output may be NULL.
 * For tests of that unwinding, two environment variables inject failures: LSX_TEST_FAIL_ALLOC=k
 * makes the k-th device allocation counted from when the variable was set (or last changed)
 * fail with LSX_E_OOM, and LSX_TEST_FAIL_EIG=1 makes plan creation report that the fibre
 * eigensolver did not converge (LSX_E_EIG).
 */
lsx_status lsx_live_buffers(int64_t* count, int64_t* bytes);

/*
 * lsx_system_create -- the problem statement (Sec. 2) and its lifted cutoff set (Sec. 3).
 *
 *  d            layer dimension, 1 or 2.
 *  A1, A2       d*d lattice matrices, column-major (column k = primitive vector k):
 *               R_j = { A_j n : n in Z^d } (Sec. 2).  Must be invertible.
 *  Ec           energy cutoff > 0 (Sec. 3).
 *  cutoff       LSX_CUTOFF_BALL:    I = {(m,n) : |G1m|^2 + |G2n|^2 <= 2 Ec}
 *               LSX_CUTOFF_PRODUCT: I = I1 x I2 with |G1m|^2 <= 2Ec, |G2n|^2 <= 2Ec (Sec. 3)
 *               where G_jm = 2 pi A_j^{-T} m.  A point is kept when
 *               s <= 2 Ec (1 + 1e-12), s = sum_k (G1m)_k^2 + sum_k (G2n)_k^2.
 *  nv1, v1_idx, v1_re, v1_im
 *               Fourier coefficients v^(1)_m of the layer-1 potential (eq. 2.2):
 *               nv1 entries, v1_idx is nv1*d int32 (entry e has index
 *               v1_idx[e*d .. e*d+d-1]), value v1_re[e] + i v1_im[e].  Indices must
 *               be distinct; the set must be Hermitian (v_{-m} = conj(v_m) within
 *               1e-14 * max|v|), otherwise LSX_E_NOT_HERMITIAN.  nv1 may be 0.
 *  nv2, ...     same for layer 2.
 *  out          receives the new handle.
 *
 * Host-only: enumerates I in canonical (lexicographic in m_1..m_d, n_1..n_d)
 * order and builds the fibre tables; touches no GPU.
 */
lsx_status lsx_system_create(int32_t d, const double* A1, const double* A2, double Ec, int32_t cutoff,
                             int32_t nv1, const int32_t* v1_idx, const double* v1_re, const double* v1_im,
                             int32_t nv2, const int32_t* v2_idx, const double* v2_re, const double* v2_im,
                             lsx_system** out);

/*
 * lsx_system_create_layers -- a system of nlayers = 2 or 3 periodic layers (Sec. 2; the
 * lifting of Sec. 3 with one index block per layer).
 *
 *  A            nlayers pointers to d*d lattice matrices (column-major, as above).
 *  nv, v_idx, v_re, v_im
 *               nlayers entries each: the Fourier coefficients of layer j's potential in
 *               the format of lsx_system_create (nv[j] may be 0; the arrays must not be NULL).
 *  cutoff       LSX_CUTOFF_BALL:    sum_j |G_j m_j|^2 <= 2 Ec
 *               LSX_CUTOFF_PRODUCT: |G_j m_j|^2 <= 2 Ec for every j (same tolerance as above).
 *
 * The lifted index of a row is (m_1, ..., m_nlayers), each m_j in Z^d; canonical order is
 * lexicographic in that tuple, and V^j couples only m_j.  A layer-j fibre fixes every block
 * but m_j; fibres are ordered by their fixed blocks (lexicographic, layer order), rows
 * ascending, so the last layer's fibres are contiguous runs of the canonical order.  With
 * nlayers = 2 this is lsx_system_create.  Three-layer systems take every scheme, the
 * deterministic entry points (plans, states, lsx_step, lsx_fibre_pass, lsx_phase,
 * lsx_observables) and batches; samplers and the semi-implicit step reject them with
 * LSX_E_INVALID.  Index entries beyond +-511 (three layers, d = 2) are rejected.
 */
lsx_status lsx_system_create_layers(int32_t d, int32_t nlayers, const double* const* A, double Ec, int32_t cutoff,
                                    const int32_t* nv, const int32_t* const* v_idx, const double* const* v_re,
                                    const double* const* v_im, lsx_system** out);

/*
 * lsx_system_create_blocks -- a lifted system whose layers may share index blocks (Example 3
 * of Sec. 5: a direction that is periodic for every layer is lifted once and coupled by every
 * layer's potential).
 *
 *  D            physical dimension, 1 or 2.
 *  nblocks      1 to 4 index blocks; block b is an integer vector m_b of block_dim[b] (1 or 2)
 *               entries with embedding R[b] (D x block_dim[b], column-major: column c is the
 *               wavevector of entry c), so a lifted index (m_0, ..., m_{B-1}) is the plane
 *               wave with K = sum_b R_b m_b.  At most 6 index entries in total.
 *  group        cutoff group of every block (numbered 0, 1, ... without gaps): a lifted index
 *               is kept when sum_{b in g} |R_b m_b|^2 <= 2 Ec (1 + 1e-12) for every group g.
 *  nlayers      2 or 3 layers; layer j couples the blocks layer_first[j] .. layer_first[j] +
 *               layer_count[j] - 1, and the last layer must couple the last block.
 *  nv, v_idx, v_re, v_im
 *               layer j's Fourier coefficients as in lsx_system_create, each index having
 *               as many entries as the layer's blocks together: V^j maps (m) to (m') when
 *               the coupled entries differ by the coefficient's index and all others agree.
 *
 * H = kappa D + sum_j ((1 - kappa)/nlayers D + V^j).  Canonical order is lexicographic in
 * (m_0, ..., m_{B-1}); a layer-j fibre fixes every entry outside the layer's blocks.  Plans,
 * states, lsx_step, lsx_fibre_pass, lsx_phase and lsx_observables accept these systems as
 * any other, with every scheme, and in batches; samplers and the semi-implicit step reject them.
 * Host-only; touches no GPU.
 */
lsx_status lsx_system_create_blocks(int32_t D, int32_t nblocks, const int32_t* block_dim, const double* const* R,
                                    const int32_t* group, double Ec, int32_t nlayers, const int32_t* layer_first,
                                    const int32_t* layer_count, const int32_t* nv, const int32_t* const* v_idx,
                                    const double* const* v_re, const double* const* v_im, lsx_system** out);

/* Number of layers and, if nfibres is not NULL, the fibre count of every layer (nlayers
 * int64 entries). */
lsx_status lsx_system_layers(const lsx_system* sys, int32_t* nlayers, int64_t* nfibres);

/* Sizes: N = |I|, and the number of fibres of layers 1 and 2.  Any output pointer may be NULL. */
lsx_status lsx_system_size(const lsx_system* sys, int64_t* N, int64_t* nfibres1, int64_t* nfibres2);

/* The lifted index set: mn is N*S int32 (host), row i the lifted index of coefficient i: S =
 * nlayers*d entries (m_1, ..., m_nlayers) for systems built from lattices (for two layers
 * (m_1..m_d, n_1..n_d)), the concatenated blocks for lsx_system_create_blocks. */
lsx_status lsx_index_get(const lsx_system* sys, int32_t* mn);

/*
 * Fibre tables of one layer (Sec. 3, block structure of V^1 and of the permuted V^2).
 * Layer 1: one fibre per n, rows {i : n_i = n}; layer 2: one fibre per m, rows {i : m_i = m}.
 * Fibres are ordered by their key (lexicographic), rows ascending.
 *  ptr   nfibres+1 int32 (host): rows of fibre f are rows[ptr[f] .. ptr[f+1]-1].  May be NULL.
 *  rows  N int32 (host).  May be NULL.
 */
lsx_status lsx_fibre_get(const lsx_system* sys, int32_t layer, int32_t* ptr, int32_t* rows);

/* Frees the system.  LSX_E_STATE if plans built on it are still alive. */
lsx_status lsx_system_destroy(lsx_system* sys);

/*
 * Point symmetries of a lattice-built system (host only): rotations R of the plane (multiples
 * of 30 degrees; in 1D, x -> -x) with R B_j = B_j M_j for an integer matrix M_j on every layer j
 * (B_j = 2 pi A_j^{-T}, Sec. 2), every potential coefficient at M_j m equal to the one at m
 * (eq. 2.2) and the lifted index set mapped onto itself (Sec. 3).  *nsym receives their number
 * (the identity not counted); M, if not NULL, receives nsym * nlayers row-major d x d int32
 * matrices M_j, symmetry-major.  Plans share fibre propagators over them (lsx_plan_sharing).
 * Systems built from shared blocks report none.
 */
lsx_status lsx_system_symmetries(const lsx_system* sys, int32_t* nsym, int32_t* M);

/*
 * lsx_plan_create -- one-time precompute of the fibre propagators on the GPU.
 *
 * Splitting (Sec. 4.2, App. A) of H = D + V^1 + V^2 (eq. 3.5) with a kinetic
 * share kappa in [0, 1]:  H = kappa D + H_1 + H_2,  H_j = (1-kappa)/2 D + V^j.
 * kappa = 0 is the paper's layer split; kappa > 0 moves that share of D into an
 * elementwise phase exp(-i kappa t |G1m+G2n|^2 / 2).
 * For every fibre the FP64 fibre Hamiltonian is assembled and diagonalised on the
 * device (batched Jacobi), and P(t) = U exp(-i t Lambda) U^H is formed for the
 * sub-step lengths the scheme needs:
 *   LSX_LIE, LSX_LIE_BE       : F1(tau), Phase(kappa tau), F2(tau)                      per step
 *   LSX_STRANG, LSX_STRANG_CN : F1(tau/2), Phase(kappa tau/2), F2(tau), Phase(kappa tau/2), F1(tau/2)
 *   LSX_YOSHIDA4              : S(g1 tau) S(g0 tau) S(g1 tau) with S the Strang step,
 *                               g1 = 1/(2 - 2^(1/3)), g0 = 1 - 2 g1 (the symmetric triple jump of
 *                               Yoshida's higher-order splittings, which the paper points to in
 *                               App. A); the adjacent F1 halves are merged.
 * The sub-step lengths a plan holds ("slots", used by lsx_plan_propagator, lsx_fibre_pass,
 * lsx_phase and lsx_sampler_increments):
 *   Lie, BE-Lie     : layer 1 {0: tau}, layer 2 {0: tau}, phase {0: tau}
 *   Strang, CN      : layer 1 {0: tau, 1: tau/2}, layer 2 {0: tau}, phase {0: tau, 1: tau/2}
 *   Yoshida         : layer 1 {0: g1 tau, 1: g1 tau/2, 2: (g1+g0) tau/2},
 *                     layer 2 {0: g1 tau, 2: g0 tau}, phase {0: g1 tau/2, 1: g0 tau/2}
 * Three-layer systems, with H_j = (1 - kappa)/3 D + V^j:
 *   Lie, BE-Lie     : F1(tau), F2(tau), Phase(kappa tau), F3(tau); every layer {0: tau},
 *                     phase {0: tau}
 *   Strang, CN      : F1(tau/2), F2(tau/2), Phase(kappa tau/2), F3(tau), Phase(kappa tau/2),
 *                     F2(tau/2), F1(tau/2); layer 1 {0: tau, 1: tau/2}, layer 2 {1: tau/2},
 *                     layer 3 {0: tau}, phase {0: tau, 1: tau/2} (CN steps are not merged)
 *   Yoshida         : the three-layer Strang steps of g1 tau, g0 tau, g1 tau; layer 1 as for two
 *                     layers, layer 2 {0: g1 tau/2, 1: g0 tau/2}, layer 3 {0: g1 tau, 2: g0 tau},
 *                     phase {0: g1 tau/2, 1: g0 tau/2}
 * with F(t) = f(H_j) per fibre and, per eigenvalue lambda, f = exp(-i t lambda) (exact
 * flows), 1/(1 + i t lambda) (backward Euler) or (1 - i t lambda/2)/(1 + i t lambda/2)
 * (Crank-Nicolson; for t = tau/2 this is (4I + i tau H)^{-1}(4I - i tau H) of eq. 4.6).
 * With kappa = 1 fibres whose index windows coincide up to a translation share one
 * eigendecomposition and one stored propagator.
 * precision    LSX_FP64: complex128 propagators, FP64 MFMA.
 *              LSX_MIX_FP32: P = diag(d) + E with d complex128 and E complex64, FP32 MFMA
 *                 on E with FP32 accumulation, FP64 diagonal term and FP64 carried state.
 *              LSX_MIX_BF16X3: as MIX_FP32 but E and the state operand are each split
 *                 into three bf16 terms; six cross products on BF16 MFMA, FP32 accumulation.
 *  tau          time step (any finite nonzero value; negative runs backwards).
 *  stream       stream for the precompute; the call synchronises it before returning.
 * Errors: LSX_E_INVALID (scheme/precision/kappa), LSX_E_EIG, LSX_E_OOM, LSX_E_HIP.
 */
lsx_status lsx_plan_create(lsx_system* sys, double tau, int32_t scheme, double kappa, int32_t precision,
                           void* stream, lsx_plan** out);

/*
 * Copies one fibre propagator P(t) back to the host as a dense L*L complex matrix
 * (row-major, interleaved; L = fibre length), with t the sub-step length of slot `half`
 * (0: tau, 1: tau/2 for Lie/Strang; see lsx_plan_create).  For mixed plans this is d + E as
 * stored (E rounded to the plan's precision).  LSX_E_INVALID if the plan holds no such
 * propagator.  Synchronous.
 */
lsx_status lsx_plan_propagator(const lsx_plan* plan, int32_t layer, int32_t half, int32_t fibre,
                               double* out, void* stream);

/*
 * Propagator sharing of a plan: *ndistinct = number of distinct fibre propagators the plan
 * stores per slot for `layer` (1 .. nlayers), *nsym = number of point symmetries other than the
 * identity they are shared over.  With kappa = 1, fibres whose index windows coincide up to a
 * translation share one propagator.  With kappa < 1 (every scheme), rotations of the plane (or
 * x -> -x in 1D) that map every layer's reciprocal lattice, potential and the lifted index set
 * onto themselves (for the twisted triangular bilayer the six rotations by multiples of 60
 * degrees) map fibre Hamiltonians onto row permutations of one another (eq. 3.6), so one
 * propagator serves each orbit (Sec. 3 block structure; LSX_SYMMETRY=0 turns this off).
 * Results are the same up to rounding either way; lsx_plan_propagator returns every fibre's
 * propagator in the row order of lsx_fibre_get.  Outputs may be NULL.
 */
lsx_status lsx_plan_sharing(const lsx_plan* plan, int32_t layer, int32_t* ndistinct, int32_t* nsym);

/*
 * Band-limited products.  Over one step an entry P_ab of a fibre propagator arises only from
 * chains of potential couplings linking rows a and b (eq. 3.6), each link of order t|v|, so
 * the entries fall off fast away from the diagonal.  At plan creation the library records,
 * for every block of 16 propagator rows, the range of column chunks (4 columns; 32 for
 * LSX_MIX_BF16X3) that hold an entry with |Re| + |Im| >= tol in any of the plan's slots, and
 * the fibre passes multiply only those chunks.  The entries left out change a pass by at most
 * L tol relative to the state (L the fibre length).  Default tol: 2^-53 for LSX_FP64 (the unit
 * roundoff: a change of the order of the pass's own rounding bound and of the accuracy of the
 * computed propagator entries), 2^-44 for the mixed precisions (far below their FP32
 * rounding); lsx_plan_desc.band_tol chooses another, and the environment variable
 * LSX_BAND_TOL overrides the default of lsx_plan_create (0: dense products).
 * lsx_plan_band: *tol = the tolerance in use (0: dense), *kept = complex multiply-adds per state
 * column of one pass of `layer` over all its fibres (rows times band width, inside the fibres),
 * *dense = the same for dense products (sum of L^2), *stored_kept = the propagator entries
 * inside the bands of the propagators the plan stores (fibres that share a propagator, see
 * lsx_plan_sharing, count once: the entries a pass must read at least once), *stored_rows = the
 * rows of the stored propagators (the diagonals a mixed pass reads).  Outputs may be NULL.
 * Host only.
 */
lsx_status lsx_plan_band(const lsx_plan* plan, int32_t layer, double* tol, int64_t* kept, int64_t* dense,
                         int64_t* stored_kept, int64_t* stored_rows);
/* The band of each 16-row block rb of one fibre (fibre order of lsx_fibre_get): lo_hi[2 rb] and
 * lo_hi[2 rb + 1] = first and one past the last fibre position whose column the pass multiplies
 * for those rows (multiples of 4, or of 32 for LSX_MIX_BF16X3; the padded fibre length at most).
 * lo_hi holds 2 ceil(L / 16) int32.  Host only. */
lsx_status lsx_plan_fibre_band(const lsx_plan* plan, int32_t layer, int32_t fibre, int32_t* lo_hi);

/* Frees the plan.  LSX_E_STATE if states built on it are still alive. */
lsx_status lsx_plan_destroy(lsx_plan* plan);

/*
 * lsx_state_create -- W wavepackets on the device, c[N][W] complex128.
 *  dev_ptr   NULL: the library allocates the array (owned by the state).
 *            non-NULL: a caller-owned device array of N*W complex doubles (16-byte
 *            aligned) that the state wraps; the caller keeps it alive until
 *            lsx_state_destroy.  Its contents are the state.
 * The library also allocates one same-size work array per state (ping-pong
 * target of the fibre passes) and small reduction buffers.
 */
lsx_status lsx_state_create(lsx_plan* plan, int32_t W, void* dev_ptr, lsx_state** out);

/* Host <-> device copies of the whole state, host layout identical to the device one
 * ([N][W] interleaved complex).  Stream-ordered; download synchronises the stream. */
lsx_status lsx_state_upload(lsx_state* st, const double* host, void* stream);
lsx_status lsx_state_download(lsx_state* st, double* host, void* stream);

/* Device address of the state array c[N][W].  For a wrapped state this is always the
 * caller's pointer.  A library-owned state keeps two arrays and may swap their roles
 * after a step or pass, so query the address again after such calls. */
lsx_status lsx_state_device_ptr(const lsx_state* st, void** dev_ptr);

/*
 * Tile shape chosen for the fibre passes of `layer` (1 .. nlayers) of this state: each
 * workgroup covers 16*nb columns and either 16 output rows with ks > 0 waves splitting the
 * fibre length, or (ks = -2, -4 or -8, mixed paths) -ks consecutive 16-row blocks, one per wave,
 * that share the state operand staged once per workgroup in LDS (each wave multiplies only its
 * own row block's band, see lsx_plan_band; FP32 needs -ks <= 4 nb, BF16x3 nb <= 2).  For W = 1
 * (matrix-vector passes) ks < 0 means 64 output rows, one per lane, with -ks waves splitting
 * the fibre length, and nb = 8 tiles that multiply the fibres sharing a
 * stored propagator together (lsx_state_set_tuning).  At creation every candidate shape is
 * timed on the state's own size
 * (LSX_AUTOTUNE=0 disables, LSX_NB / LSX_KS force a shape); pass_us is the measured
 * time of one pass with the chosen shape (0 if nothing was timed).  The single-pass winner and
 * runner-up of each layer are then compared on the step-like cycle described at
 * lsx_state_store_mode, which keeps whichever makes the cycle faster.  For the ks > 0 shapes of
 * the FP64 and mixed FP32 paths the candidates also differ in how many groups of k-steps each
 * wave keeps in flight (one or two; LSX_PREFETCH=1 / 2 / 4 forces it, a forced shape uses 2),
 * which changes the summation order, so the rounding, of the pass.  Outputs may be NULL.
 */
lsx_status lsx_state_tuning(const lsx_state* st, int32_t layer, int32_t* nb, int32_t* ks, double* pass_us);

/* Groups of k-steps each wave keeps in flight in the fibre passes of `layer` (1 .. nlayers),
 * for the ks > 0 shapes of the FP64 and mixed FP32 paths: 1 or 2, chosen at creation by the
 * tile tuner's single passes and then kept or flipped by the step-like cycle timed for the
 * store mode (lsx_state_store_mode); 0 where the library default applies (2, or LSX_PREFETCH;
 * also every other shape and a forced shape). */
lsx_status lsx_state_prefetch(const lsx_state* st, int32_t layer, int32_t* groups);

/*
 * Store mode chosen for the outputs of this state's fibre passes: *nontemporal = 1 when they
 * are streamed out of the writing XCD's L2 (non-temporal stores), 0 for ordinary stores.  A
 * step's next pass reads the output in its own layer's fibre order, mostly on other XCDs, so
 * the faster mode depends on the state's size relative to the caches.  At creation, after the
 * tile shapes, a cycle of passes over the layers in step order is timed with both modes, for
 * the tile tuner's choice and, one layer at a time, for that layer's alternatives (the other
 * prefetch depth where one was tuned, see lsx_state_prefetch, and the single-pass runner-up
 * shape); the fastest combination is kept.  The cycle runs between the work array and a
 * temporary array of the state's size (the state is not read or written; without memory for
 * the temporary array the mode stays 0).  cycle_us[0], [1] are the best cycle times measured
 * with each mode (0 if not timed).  LSX_NT=0 / 1 forces a mode;
 * LSX_AUTOTUNE=0 and W = 1 (matrix-vector passes) keep 0.  The mode changes no result: both
 * give bit-identical states.  Outputs may be NULL.
 */
lsx_status lsx_state_store_mode(const lsx_state* st, int32_t* nontemporal, double* cycle_us);

/*
 * Pinning the tuned shape, for bitwise-repeatable runs.  The tuners above choose from timings,
 * which vary from run to run, and a different shape or prefetch depth changes the summation
 * order of a pass.  Reading a state's choice (lsx_state_tuning, lsx_state_prefetch,
 * lsx_state_store_mode) and setting it on another state, in this or a later process, makes the
 * two step bit for bit alike.
 * lsx_state_set_tuning: tile shape (nb, ks) and k-step groups in flight (`groups`, 0 for the
 *   library default) of `layer`'s passes; the tile list is rebuilt on the host and uploaded
 *   (synchronous).  Available shapes: W = 1: nb = 1 and ks in {1, 2, 4}, or {-1, -2, -4, -8}
 *   (tiles of 64 rows, one row per lane), groups = 0; nb = 8 with the same ks: orbit tiles, which multiply up to
 *   eight fibres that share one stored propagator (lsx_plan_sharing) with one load of each
 *   propagator chunk and give the same result as nb = 1 with that ks (LSX_E_INVALID on a layer
 *   where no fibre shares).  W > 1: nb in {1, 2, 4} with 16 nb <= W rounded up to 16; ks in
 *   {1, 2, 4} with groups 0, or 1 or 2 for LSX_FP64 / LSX_MIX_FP32; or ks in {-2, -4, -8} for
 *   the mixed paths (-ks <= 4 nb for LSX_MIX_FP32, nb <= 2 for LSX_MIX_BF16X3), groups 0.
 *   Anything else is LSX_E_INVALID and leaves the state unchanged.  lsx_state_tuning then
 *   reports pass_us = 0.
 * lsx_state_set_store_mode: 0 ordinary, 1 non-temporal output stores (LSX_E_INVALID otherwise).
 * Neither call touches the state's values.  Not while a step on the state is in flight.
 */
lsx_status lsx_state_set_tuning(lsx_state* st, int32_t layer, int32_t nb, int32_t ks, int32_t groups);
lsx_status lsx_state_set_store_mode(lsx_state* st, int32_t nontemporal);

lsx_status lsx_state_destroy(lsx_state* st);

/*
 * lsx_step -- advances the state by exactly nsteps * tau with the plan's scheme
 * (App. A compositions; with exact flows the Strang half-steps of consecutive steps inside
 * one call are merged, F1(tau/2) F1(tau/2) = F1(tau), and so are the adjacent F1 sub-steps
 * of the Yoshida scheme; Crank-Nicolson steps are applied unmerged).  nsteps >= 0.
 * Stream-ordered.  Where the passes are launch-bound (every layer's tuned pass at most
 * 20 us) and a call repeats the step body often enough, the library captures its passes
 * once into HIP graphs and replays them: graphs of about 512 passes for the bulk of the
 * call, then halved sizes down to about 32 passes for the remainder (LSX_GRAPH_PASSES,
 * LSX_GRAPH_MIN_PASSES), the passes short of the smallest launched directly.  The graphs are
 * kept with the state, one per size and arrangement of its two arrays, up to 16 (the least
 * recently used is replaced, after a device synchronisation), and rebuilt after
 * lsx_state_set_tuning / lsx_state_set_store_mode; the launches and results are the same as
 * without.  LSX_GRAPH=1 / 0 forces graphs on / off.
 * While the caller's stream is itself being captured, every pass is launched on it
 * directly.
 */
lsx_status lsx_step(lsx_plan* plan, lsx_state* st, int64_t nsteps, void* stream);

/*
 * lsx_fibre_pass -- one layer sub-step on its own: c[rows_f] <- P_f(t) c[rows_f]
 * for every fibre f of `layer` (Alg. 2 steps 1/2 with exact fibre flows), with
 * t the length of slot `half` (0: tau, 1: tau/2 for Lie/Strang; see lsx_plan_create),
 * applied `count` >= 0 times back to back (one kernel launch each; count > 1 is used to
 * time the pass).  Stream-ordered.
 */
lsx_status lsx_fibre_pass(lsx_plan* plan, lsx_state* st, int32_t layer, int32_t half, int32_t count,
                          void* stream);

/*
 * lsx_phase -- kinetic sub-step c_i <- exp(-i kappa t |G1m+G2n|^2 / 2) c_i, with
 * t the plan's phase slot `half` (0: tau, 1: tau/2 for Lie/Strang; see lsx_plan_create)
 * and the plan's kappa (Alg. 3 step 1 with kinetic share kappa).  A no-op when kappa = 0.
 * Stream-ordered.
 */
lsx_status lsx_phase(lsx_plan* plan, lsx_state* st, int32_t half, void* stream);

/*
 * lsx_observables -- FP64 reductions on the device, result copied to `out` (host).
 * mask selects, in this order of output blocks:
 *   LSX_OBS_MASS          N_w = sum_i |c_iw|^2  (eq. 2.3 via the orthonormality 3.1)
 *   LSX_OBS_ENERGY        E_w = sum_i 1/2 |K_i|^2 |c_iw|^2 + Re c_w^H (V^1 + V^2 [+ V^3]) c_w (eq. 2.4)
 *   LSX_OBS_FIBRE_MASS_1  [f][w] partial masses over layer-1 fibres
 *   LSX_OBS_FIBRE_MASS_2  [f][w] partial masses over layer-2 fibres
 *   LSX_OBS_FIBRE_MASS_3  [f][w] partial masses over layer-3 fibres (three-layer systems)
 * Deterministic (fixed reduction order).  Synchronises the stream.
 * LSX_E_NONFINITE if any requested value is NaN/Inf (out is still written).
 */
lsx_status lsx_observables(lsx_plan* plan, lsx_state* st, uint32_t mask, double* out, void* stream);

/*
 * lsx_observables_noalloc -- lsx_observables for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  It
 * calls no hipMalloc, hipFree or allocating library routine.
 *  dev_c    caller-owned device array c[N][W] complex128 (N of the plan's system), read only.
 *  W        1 .. 65536 wavepackets (and at most the plan's max_wavepackets, if set).
 *  mask     as for lsx_observables; the output blocks follow in the same order.
 *  dev_out  caller-owned DEVICE array that receives the requested blocks (W doubles for mass
 *           and energy, nfibres_j * W for fibre masses), stream-ordered; nothing is copied to
 *           the host and the stream is not synchronised.  Non-finite values are not checked
 *           (the results never reach the host here).
 * The mass and energy reductions keep their partial sums in a static scratch array of 2^20
 * doubles (8 MiB) per GPU, held until the process ends; a call needs
 * W * min(1024, ceil(N / 256)) of them and is refused beyond that with LSX_E_INVALID (fibre
 * masses alone need none).  Every partial is written before it is read within a call, so no
 * part of the array has to start at zero.  All calls on one GPU share the array: calls that
 * overlap on one GPU (different streams or threads) race.  Same kernels, block count and
 * fixed reduction order as lsx_observables, so the values are identical.
 */
lsx_status lsx_observables_noalloc(lsx_plan* plan, const void* dev_c, int32_t W, uint32_t mask, double* dev_out,
                                   void* stream);

/*
 * Descriptor form of the boundary.  The same problem statement (Sec. 2: lattices R_j = A_j Z^d
 * and the Fourier coefficients of the layer potentials, eq. 2.2; Sec. 3: the cutoff Ec and its
 * lifted set) and the same plan parameters (tau, scheme of App. A / Alg. 2 / eq. 4.6, kinetic
 * share, precision) gathered in two structs, with calls named for what they return.  Each is a
 * thin wrapper of the flat-argument call named beside it, with that call's argument meaning,
 * layout, ownership and errors.
 *   lsx_system_desc: d (1 or 2); A1, A2 column-major d x d (entries past d*d ignored); Ec;
 *     cutoff (LSX_CUTOFF_BALL / LSX_CUTOFF_PRODUCT); per layer j = 0, 1: nv[j] coefficients,
 *     v_idx[j] (nv[j]*d int32), v_re[j], v_im[j].
 *   lsx_plan_desc: tau, scheme, kappa, precision as for lsx_plan_create; max_wavepackets > 0
 *     makes lsx_state_create / lsx_state_wrap refuse W above it (LSX_E_INVALID); 0: no limit;
 *     band_tol (see lsx_plan_band): 0 the default for the precision, < 0 dense products,
 *     > 0 this tolerance; NaN is LSX_E_INVALID.
 * lsx_system_create_desc = lsx_system_create (host only).
 * lsx_index_size: *N = |I| (as lsx_system_size's N).
 * lsx_fibre_info: number of fibres of `layer` (1 .. nlayers) and, if `lengths` is not NULL,
 *   their lengths (nfibres int32, fibres in the order of lsx_fibre_get).
 * lsx_plan_create_desc = lsx_plan_create (one-time precompute, synchronises the stream).
 * lsx_state_wrap = lsx_state_create with a caller-owned device array (dev_ptr must not be
 *   NULL): c[N][W] complex128, 16-byte aligned, kept alive by the caller until
 *   lsx_state_destroy.  The host layout of lsx_state_upload / download is [N][W] as on the
 *   device (W innermost), so that upload and download are plain copies.
 */
typedef struct {
  int32_t d;
  double A1[4], A2[4];
  double Ec;
  int32_t cutoff;
  int32_t nv[2];
  const int32_t* v_idx[2];
  const double* v_re[2];
  const double* v_im[2];
} lsx_system_desc;
typedef struct {
  double tau;
  int32_t scheme;
  double kappa;
  int32_t precision;
  int32_t max_wavepackets;
  double band_tol;
} lsx_plan_desc;
lsx_status lsx_system_create_desc(const lsx_system_desc* desc, lsx_system** out);
lsx_status lsx_index_size(const lsx_system* sys, int64_t* N);
lsx_status lsx_fibre_info(const lsx_system* sys, int32_t layer, int64_t* nfibres, int32_t* lengths);
lsx_status lsx_plan_create_desc(lsx_system* sys, const lsx_plan_desc* desc, void* stream, lsx_plan** out);
lsx_status lsx_state_wrap(lsx_plan* plan, int32_t W, void* dev_ptr, lsx_state** out);

/*
 * Batched systems -- several independent (plan, state) pairs advanced together: every
 * fibre pass of the batch is ONE grouped kernel launch over the tiles of all systems
 * (fibres of uneven lengths, systems of different cutoffs, lattices, W); where the grouped
 * passes are launch-bound (as for lsx_step), the repeated part of the step sequence is
 * captured once in a HIP graph (about 128 passes, repetitions short of a whole graph run
 * directly) and replayed.
 *
 * lsx_batch_create: plans[i] and states[i] (i < n) must match (states[i] created on
 *   plans[i]); all plans must share the scheme, the precision and the number of layers;
 *   states must be all W = 1 or all W >= 2.  The tile shape and the launch mode of every layer's pass are
 *   autotuned on the whole batch: one workgroup per tile (the hardware dispatcher balances
 *   the uneven tiles), or a persistent grid of the resident capacity that walks the
 *   XCD-interleaved tile list with a static stride, or one that claims tiles from per-XCD
 *   queues on device counters (cleared by the last workgroup of each launch, so replayed
 *   graphs need no memset).  All three give bit-identical results for one tile shape.  For
 *   the FP64 and mixed FP32 paths the candidates also differ in the groups of k-steps each
 *   wave keeps in flight (one or two, as for states; LSX_PREFETCH is not applied here, and a
 *   forced shape keeps two).
 *   Plans and states must outlive the batch (destroying a state that is in a batch returns
 *   LSX_E_STATE).  While a batch step is in flight no other call may use its states.
 * lsx_batch_step: advances every state by nsteps * tau_i with its plan's scheme, exactly
 *   as lsx_step would (bit-for-bit up to the tile shape's summation order).  Stream-ordered.
 * lsx_batch_tuning: tile shape, measured pass time and launch mode (0 one workgroup per tile,
 *   1 persistent with tile queues, 2 persistent with a static stride) of `layer` for the whole
 *   batch.  Any output pointer may be NULL.
 */
typedef struct lsx_batch lsx_batch;
lsx_status lsx_batch_create(lsx_plan* const* plans, lsx_state* const* states, int32_t n, lsx_batch** out);
lsx_status lsx_batch_step(lsx_batch* batch, int64_t nsteps, void* stream);
lsx_status lsx_batch_tuning(const lsx_batch* batch, int32_t layer, int32_t* nb, int32_t* ks, double* pass_us,
                            int32_t* launch_mode);
lsx_status lsx_batch_destroy(lsx_batch* batch);

/* ================================================================ semi-implicit, random batch and
 * stochastic layer splitting
 *
 * lsx_si_step -- nsteps steps of the semi-implicit method (Alg. 1, Sec. 4.1):
 *     c <- (I + i tau D)^{-1} (c - i tau V^1 c - i tau V^2 c),   D = diag(|G1m + G2n|^2 / 2),
 *   with the plan's tau.  The potentials act through the neighbour stencil of eq. 3.6 in FP64;
 *   the plan's scheme, kappa and precision do not enter.  Stream-ordered; uses the state's
 *   work array.
 */
lsx_status lsx_si_step(lsx_plan* plan, lsx_state* st, int64_t nsteps, void* stream);

typedef struct lsx_sampler lsx_sampler;
typedef struct lsx_mlp lsx_mlp;

/*
 * lsx_sampler_create -- workspace of the stochastic steps of (plan, st).  Every wavepacket
 *   (column) of the state samples on its own.
 *   p1, p2  fibres drawn per wavepacket for each layer-1 / layer-2 sub-step, >= 0.  For
 *           lsx_ss_step, 0 makes that layer's sub-steps the full deterministic pass (the
 *           fallback); lsx_rb_step needs 1 <= p_j <= nfibres_j.
 *   eps     in [0, 1]: uniform share of the importance proposal (keeps every q_f > 0).
 *   Layers with more than 2048 fibres are rejected (LSX_E_INVALID).  The sampler must be
 *   destroyed before its state and plan (LSX_E_STATE otherwise).
 */
lsx_status lsx_sampler_create(lsx_plan* plan, lsx_state* st, int32_t p1, int32_t p2, double eps,
                              lsx_sampler** out);
/* Attach the proposal network (NULL: uniform proposal).  Its input count must be d + 3.
 * The network must outlive the sampler's use of it (lsx_mlp_destroy refuses while attached). */
lsx_status lsx_sampler_set_mlp(lsx_sampler* sm, lsx_mlp* mlp);
lsx_status lsx_sampler_destroy(lsx_sampler* sm);

/*
 * lsx_rb_step -- nsteps steps of the random batch method (Alg. 4): the step of lsx_si_step
 *   with V^1 applied only on p1 layer-1 fibres and V^2 only on p2 layer-2 fibres, chosen per
 *   wavepacket uniformly without replacement and scaled by nfibres_j / p_j (the fibre counts
 *   stand for |I_2| and |I_1| of the paper).
 *   u  device array [nsteps][2][W][pmax] of uniforms in [0, 1), pmax = max(p1, p2);
 *      u[k][j-1][w][s] places the s-th pick of layer j for wavepacket w in step k by a partial
 *      Fisher-Yates shuffle (position s swaps with s + floor(u (nfibres_j - s))).
 *   Stream-ordered; the caller keeps u alive until the stream has passed the call.
 */
lsx_status lsx_rb_step(lsx_sampler* sm, const double* u, int64_t nsteps, void* stream);

/*
 * lsx_ss_step -- nsteps steps of stochastic layer splitting: the plan's Lie or Strang
 *   composition (App. A; unmerged) with every fibre sub-step F_j(t) c = c + sum_f (P_f - I) c_f
 *   replaced by the unbiased estimate
 *       c + sum_{s=1..p_j} (P_{f_s}(t) - I) c_{f_s} / (p_j q_{f_s}),
 *   the fibres f_s drawn independently per wavepacket from q = (1 - eps) softmax(z) + eps / nf
 *   (z: the attached network on lsx_sampler_features of the state entering the sub-step;
 *   uniform q without a network).  This carries the random batch idea of Alg. 4 over to the
 *   fibre flows of Alg. 2 / App. A.  Sub-steps: Lie F1(tau), F2(tau); Strang F1(tau/2),
 *   F2(tau), F1(tau/2); the kinetic phase follows F1 and F2 as in lsx_step when kappa > 0.
 *   u  device array [nsteps][nsub][W][pmax] (nsub = 2 Lie, 3 Strang): draw s of sub-step k
 *      in step n is the first fibre whose running sum of q exceeds u[n][k][w][s].
 *   Stream-ordered; uses the state's work array.
 */
lsx_status lsx_ss_step(lsx_sampler* sm, const double* u, int64_t nsteps, void* stream);

/*
 * lsx_sampler_weights -- one layer's sampling alone.  wt: device [nfibres][W] (FP64).
 *   mode 0: importance draws (weights 1/(p q_f) summed per fibre) from logits z (device
 *           [W][nfibres] FP32, NULL = uniform) with the sampler's eps and p_layer >= 1;
 *   mode 1: Alg. 4 subsets, weight nfibres / p_layer on the chosen fibres (z ignored).
 *   u: device [W][p_layer].  Stream-ordered.
 */
lsx_status lsx_sampler_weights(lsx_sampler* sm, int32_t layer, int32_t mode, const float* z, const double* u,
                               double* wt, void* stream);

/*
 * lsx_sampler_features -- inputs of the proposal network for the state's current coefficients:
 *   X device [W][nfibres][d+3] FP32, per wavepacket and fibre of `layer`: shift / Kmax (d
 *   entries), |shift / Kmax|^2, log10(max(fibre mass, 1e-30)) / 10, layer sign (-1 layer 1,
 *   +1 layer 2); shift = G2 n for the layer-1 fibre of n, G1 m for the layer-2 fibre of m
 *   (the Bloch shift of Sec. 3), Kmax = sqrt(2 Ec).  Stream-ordered.
 */
lsx_status lsx_sampler_features(lsx_sampler* sm, int32_t layer, float* X, void* stream);

/*
 * lsx_sampler_increments -- b device [W][nfibres] FP64: ||(P_f(t) - I) c_f||^2 per wavepacket
 *   and fibre of `layer`, t = the length of slot `half` (0: tau, 1: tau/2), from the plan's propagators.  The
 *   optimal proposal of a sub-step is q_f ~ sqrt(b_f); these are the network's training
 *   targets.  The state is not modified (the work array is).  Stream-ordered.
 */
lsx_status lsx_sampler_increments(lsx_sampler* sm, int32_t layer, int32_t half, double* b, void* stream);

/* ================================================================ proposal network
 *
 * A 3-layer tanh MLP of width 64 in FP32: z = w3 . tanh(W2^T tanh(W1^T x + b1) + b2) + b3 with
 * nin in [1, 8] inputs.  Flat parameter order: W1 [nin][64] row-major, b1 [64], W2 [64][64]
 * row-major, b2 [64], w3 [64], b3 (64 nin + 4289 floats).  Device arrays are the caller's.
 *
 * lsx_mlp_create     parameters and Adam moments start at zero.
 * lsx_mlp_set/get    host copies of the flat parameters (set also resets Adam; get synchronises).
 * lsx_mlp_forward    z[m] for the M rows of X [M][nin] (device).
 * lsx_mlp_backward   grad (device, nparams) = d(sum_m dz[m] z[m]) / d theta.
 * lsx_mlp_loss       normalised variance objective of groups g = rows gptr[g]..gptr[g+1]
 *                    (gptr device, ngroups + 1 entries): q = (1 - eps) softmax(z_g) + eps / n_g,
 *                    l_g = sum b/q / (sum sqrt b)^2; out (device, 2 doubles) = mean of l_g over
 *                    groups with sum b > 0 and 1 / their count; dz (device, gptr[ngroups]) =
 *                    gradient of that mean.
 * lsx_mlp_adam       one Adam step (Kingma & Ba) with gradient grad (device).
 * lsx_mlp_train_step forward, objective, backward and Adam on one batch of M rows; out as in
 *                    lsx_mlp_loss, evaluated before the update.
 * All stream-ordered except get.
 */
lsx_status lsx_mlp_create(int32_t nin, lsx_mlp** out);
lsx_status lsx_mlp_nparams(const lsx_mlp* mlp, int64_t* n);
lsx_status lsx_mlp_set(lsx_mlp* mlp, const float* theta, void* stream);
lsx_status lsx_mlp_get(const lsx_mlp* mlp, float* theta, void* stream);
lsx_status lsx_mlp_forward(const lsx_mlp* mlp, const float* X, int64_t M, float* z, void* stream);
lsx_status lsx_mlp_backward(lsx_mlp* mlp, const float* X, int64_t M, const float* dz, float* grad, void* stream);
lsx_status lsx_mlp_loss(lsx_mlp* mlp, const float* z, const double* b, const int64_t* gptr, int64_t ngroups,
                        double eps, double* out, float* dz, void* stream);
lsx_status lsx_mlp_adam(lsx_mlp* mlp, const float* grad, double lr, double beta1, double beta2, double adam_eps,
                        void* stream);
lsx_status lsx_mlp_train_step(lsx_mlp* mlp, const float* X, int64_t M, const double* b, const int64_t* gptr,
                              int64_t ngroups, double eps, double lr, double beta1, double beta2, double adam_eps,
                              double* out, void* stream);
lsx_status lsx_mlp_destroy(lsx_mlp* mlp);

#ifdef __cplusplus
}
#endif

#endif /* LSX_H */

// Host side of liblsx: geometry and lifted index set (Secs. 2-3), fibre tables,
// plan precompute driver, state management, step composer (App. A) and the C-ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "lsx_internal.h"

namespace lsx {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static lsx_status fail(lsx_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

static double env_double(const char* name, double dflt) {
  const char* v = std::getenv(name);
  return (v && *v) ? std::atof(v) : dflt;
}

// ---------------------------------------------------------------- failure injection (tests)
// LSX_TEST_FAIL_ALLOC=k makes the k-th device allocation counted from when the variable was
// set (or last changed) report LSX_E_OOM; LSX_TEST_FAIL_EIG=1 makes the fibre eigensolver
// report non-convergence.  Both exist so that the unwinding of a failed set-up can be tested
// from the host; unset, they cost one getenv per allocation or plan.
static bool test_fail_alloc() {
  static std::mutex mu;
  static std::string last;
  static long count = 0;
  const char* v = std::getenv("LSX_TEST_FAIL_ALLOC");
  std::lock_guard<std::mutex> lock(mu);
  if (!v) {
    last.clear();
    count = 0;
    return false;
  }
  if (last != v) {
    last = v;
    count = 0;
  }
  return ++count == std::atol(v);
}

// Live device buffers of the library and their bytes (diagnostics: lsx_live_buffers).
static std::atomic<int64_t> g_live_buffers{0}, g_live_bytes{0};

// ---------------------------------------------------------------- device buffer helper
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) {
      (void)hipFree(p);
      g_live_buffers--;
      g_live_bytes -= (int64_t)(n * sizeof(T));
    }
    p = nullptr;
    n = 0;
  }
  lsx_status alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    if (test_fail_alloc()) return fail(LSX_E_OOM, "injected allocation failure (LSX_TEST_FAIL_ALLOC)");
    if (hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return fail(LSX_E_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
    g_live_buffers++;
    g_live_bytes += (int64_t)(n * sizeof(T));
    return LSX_OK;
  }
  // Set-up copy from a host vector, complete on return: callers pass locals and temporaries,
  // so the copy must not outlive `v`, whatever HIP does with pageable memory.
  lsx_status upload(const std::vector<T>& v, hipStream_t s) {
    lsx_status st = alloc(v.size());
    if (st != LSX_OK) return st;
    if (!v.empty()) {
      LSX_HIP_TRY(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
      LSX_HIP_TRY(hipStreamSynchronize(s));
    }
    return LSX_OK;
  }
};

#define LSX_TRY(expr)                     \
  do {                                    \
    lsx_status st_ = (expr);              \
    if (st_ != LSX_OK) return st_;        \
  } while (0)

}  // namespace lsx

using namespace lsx;

// ================================================================ system
struct Stencil {
  std::vector<int32_t> idx;  // nv*d
  std::vector<double> re, im;
  int nv = 0;
  bool real = true;
};

struct FibreTable {
  std::vector<int32_t> ptr, rows;
  int maxL = 0;
};

// The lifted index of row i is a sequence of integer blocks (m_0, ..., m_{B-1}), block b of
// dimension dim_b with physical embedding R_b (K = sum_b R_b m_b).  Layer j's potential
// couples the contiguous index columns [lown[j], lown[j] + ldim[j]).  Systems built from
// lattices have one block per layer (the lifted index (m_1, ..., m_nl), each m_j in Z^d).
static constexpr int kMaxLayers = 3;
static constexpr int kMaxBlocks = 4;
static constexpr int kMaxIndex = 6;  // entries of a lifted index

struct lsx_system {
  int d = 1;          // layer dimension (systems built from lattices); physical dimension otherwise
  int nl = 2;         // number of layers
  bool standard = true;  // built from lattices, one block per layer
  double A[kMaxLayers][4] = {};
  double B[kMaxLayers][4] = {};  // reciprocal 2 pi A^{-T}, row-major d x d
  int S = 0;                     // entries of a lifted index
  int lown[kMaxLayers] = {}, ldim[kMaxLayers] = {};
  double Ec = 0.0;
  int cutoff = 0;
  int64_t N = 0;
  std::vector<int32_t> mn;  // N * S
  std::vector<double> K2;   // |K|^2
  Stencil pot[kMaxLayers];
  FibreTable fib[kMaxLayers];
  std::vector<int32_t> nbr[kMaxLayers];  // N * nv_j: row with layer j's columns shifted by -p, or -1
  int nplans = 0;
};

// One index block: dimension and physical embedding R (row-major D x dim).
struct BlockSpec {
  int dim = 1;
  double R[4] = {};
};

// A given column-major (A[k + d*c] = row k, column c); returns B = 2 pi A^{-T} row-major.
static bool reciprocal(int d, const double* A, double* B) {
  if (d == 1) {
    if (!(std::isfinite(A[0])) || A[0] == 0.0) return false;
    B[0] = 2.0 * M_PI / A[0];
    return true;
  }
  const double a = A[0], c = A[1], b = A[2], dd = A[3];  // [[a, b], [c, dd]]
  const double det = a * dd - b * c;
  if (!std::isfinite(det) || std::fabs(det) < 1e-300) return false;
  // A^{-1} = [[dd, -b], [-c, a]] / det ; A^{-T} = [[dd, -c], [-b, a]] / det
  B[0] = 2.0 * M_PI * dd / det;
  B[1] = 2.0 * M_PI * -c / det;
  B[2] = 2.0 * M_PI * -b / det;
  B[3] = 2.0 * M_PI * a / det;
  return true;
}

// All integer vectors m of a block with |R m|^2 <= lim (R row-major D x dim, full column
// rank), lexicographic order, and their |R m|^2.  |m_k| <= |row_k(R^+)| |R m| with
// |row_k(R^+)|^2 = ((R^T R)^{-1})_kk bounds the search.  False if R^T R is singular.
static bool block_candidates(int D, const BlockSpec& b, double lim, std::vector<int32_t>& out,
                             std::vector<double>& s2) {
  const int dim = b.dim;
  double G[4] = {};
  for (int p = 0; p < dim; ++p)
    for (int q = 0; q < dim; ++q)
      for (int k = 0; k < D; ++k) G[p * dim + q] += b.R[k * dim + p] * b.R[k * dim + q];
  double Ginv_diag[2];
  if (dim == 1) {
    if (!(G[0] > 0.0) || !std::isfinite(G[0])) return false;
    Ginv_diag[0] = 1.0 / G[0];
  } else {
    const double det = G[0] * G[3] - G[1] * G[2];
    if (!(det > 1e-300 * std::max(1.0, G[0] * G[3])) || !std::isfinite(det)) return false;
    Ginv_diag[0] = G[3] / det;
    Ginv_diag[1] = G[0] / det;
  }
  int bound[2] = {0, 0};
  for (int k = 0; k < dim; ++k) {
    const double x = std::floor(std::sqrt(lim * Ginv_diag[k])) + 1.0;
    if (!(x < 1e6)) return false;
    bound[k] = (int)x;
  }
  out.clear();
  s2.clear();
  auto norm2 = [&](const int32_t* m) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) {
      double g = 0.0;
      for (int c = 0; c < dim; ++c) g += b.R[k * dim + c] * m[c];
      s += g * g;
    }
    return s;
  };
  if (dim == 1) {
    for (int32_t m = -bound[0]; m <= bound[0]; ++m) {
      const double s = norm2(&m);
      if (s <= lim) {
        out.push_back(m);
        s2.push_back(s);
      }
    }
  } else {
    for (int32_t m0 = -bound[0]; m0 <= bound[0]; ++m0)
      for (int32_t m1 = -bound[1]; m1 <= bound[1]; ++m1) {
        const int32_t m[2] = {m0, m1};
        const double s = norm2(m);
        if (s <= lim) {
          out.push_back(m0);
          out.push_back(m1);
          s2.push_back(s);
        }
      }
  }
  return true;
}

// 64-bit key of an integer vector: 16 bits per entry up to 4 entries, 10 bits up to 6
// (callers check the entries fit: |v| < 2^15 or < 2^9).
static inline uint64_t pack_key(const int32_t* v, int len) {
  uint64_t k = 0;
  const int bits = len <= 4 ? 16 : 10;
  const uint64_t mask = (1ull << bits) - 1ull;
  for (int i = 0; i < len; ++i) k = (k << bits) | ((uint64_t)(int64_t)v[i] & mask);
  return k;
}

static lsx_status build_stencil(int d, int nv, const int32_t* idx, const double* re, const double* im,
                                Stencil& st, int layer) {
  if (nv < 0) return fail(LSX_E_INVALID, "negative potential size");
  if (nv > 0 && (!idx || !re || !im)) return fail(LSX_E_INVALID, "null potential array");
  st.nv = nv;
  st.idx.assign(idx, idx + (size_t)nv * d);
  st.re.assign(re, re + nv);
  st.im.assign(im, im + nv);
  double vmax = 0.0;
  for (int e = 0; e < nv; ++e) {
    if (!std::isfinite(re[e]) || !std::isfinite(im[e]))
      return fail(LSX_E_INVALID, "non-finite potential coefficient");
    vmax = std::max(vmax, std::hypot(re[e], im[e]));
    for (int k = 0; k < d; ++k)
      if (std::abs(idx[e * d + k]) > 16000) return fail(LSX_E_INVALID, "potential index out of range");
  }
  std::unordered_map<uint64_t, int> pos;
  for (int e = 0; e < nv; ++e) {
    const uint64_t key = pack_key(&idx[e * d], d);
    if (pos.count(key)) return fail(LSX_E_INVALID, "duplicate potential index in layer " + std::to_string(layer));
    pos[key] = e;
  }
  st.real = true;
  const double tol = 1e-14 * vmax;
  for (int e = 0; e < nv; ++e) {
    int32_t neg[kMaxIndex];
    for (int k = 0; k < d; ++k) neg[k] = -idx[e * d + k];
    auto it = pos.find(pack_key(neg, d));
    if (it == pos.end()) {
      if (std::hypot(re[e], im[e]) > tol)
        return fail(LSX_E_NOT_HERMITIAN, "layer " + std::to_string(layer) + ": v_{-m} missing for a nonzero v_m");
      continue;
    }
    const int o = it->second;
    if (std::fabs(re[o] - re[e]) > tol || std::fabs(im[o] + im[e]) > tol)
      return fail(LSX_E_NOT_HERMITIAN, "layer " + std::to_string(layer) + ": v_{-m} != conj(v_m)");
    if (im[e] != 0.0) st.real = false;
  }
  return LSX_OK;
}

extern "C" const char* lsx_last_error(void) { return g_err.c_str(); }

extern "C" lsx_status lsx_live_buffers(int64_t* count, int64_t* bytes) {
  if (count) *count = g_live_buffers.load();
  if (bytes) *bytes = g_live_bytes.load();
  return LSX_OK;
}

// The lifted cutoff set (Sec. 3; more than two layers as in Sec. 2; shared blocks as in
// Example 3 of Sec. 5): the candidate vectors of every block (lexicographic), combined with
// block 0 outermost, kept when every cutoff group g has sum_{b in g} |R_b m_b|^2 <= 2 Ec
// (relative tolerance 1e-12); then |K|^2, the fibres of every layer (fixing the columns the
// layer's potential does not couple) and the potentials' neighbour tables.  The stencils,
// sys->nl, sys->lown and sys->ldim are set by the caller.
static lsx_status build_lifted(lsx_system* sys, int D, int nb, const BlockSpec* blk, const int* group, double Ec) {
  const double lim = 2.0 * Ec * (1.0 + 1e-12);
  int S = 0;
  for (int b = 0; b < nb; ++b) S += blk[b].dim;
  sys->S = S;
  const int nl = sys->nl;
  std::vector<int32_t> cand[kMaxBlocks];
  std::vector<double> s2[kMaxBlocks];
  for (int b = 0; b < nb; ++b)
    if (!block_candidates(D, blk[b], lim, cand[b], s2[b]))
      return fail(LSX_E_INVALID, "block " + std::to_string(b) + " has a singular or non-finite embedding");
  // the combinations walked below bound the set from above; refuse sizes that could not be
  // indexed anyway before walking them
  double combos = 1.0;
  for (int b = 0; b < nb; ++b) combos *= (double)s2[b].size();
  if (combos > 64.0 * 2147483648.0) return fail(LSX_E_INVALID, "lifted index set too large");
  int ngroups = 0;
  for (int b = 0; b < nb; ++b) ngroups = std::max(ngroups, group[b] + 1);
  int64_t idx[kMaxBlocks] = {0, 0, 0, 0};
  // odometer over the candidate lists, last block fastest
  bool any = true;
  for (int b = 0; b < nb; ++b) any = any && !s2[b].empty();
  while (any) {
    double sum[kMaxBlocks] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b) sum[group[b]] += s2[b][idx[b]];
    bool keep = true;
    for (int g = 0; g < ngroups; ++g) keep = keep && (sum[g] <= lim);
    if (keep)
      for (int b = 0; b < nb; ++b)
        for (int k = 0; k < blk[b].dim; ++k) sys->mn.push_back(cand[b][idx[b] * blk[b].dim + k]);
    int b = nb - 1;
    while (b >= 0 && ++idx[b] == (int64_t)s2[b].size()) idx[b--] = 0;
    if (b < 0) break;
  }
  sys->N = (int64_t)sys->mn.size() / S;
  if (sys->N >= (int64_t)1 << 31) return fail(LSX_E_INVALID, "lifted index set too large");
  const int64_t N = sys->N;
  const int keymax = S <= 4 ? 32767 : 511;
  for (int32_t v : sys->mn)
    if (std::abs(v) > keymax) return fail(LSX_E_INVALID, "lifted index out of the supported range");
  sys->K2.resize(N);
  for (int64_t i = 0; i < N; ++i) {
    const int32_t* r = &sys->mn[i * S];
    double s = 0.0;
    for (int k = 0; k < D; ++k) {
      double g = 0.0;
      for (int b = 0, o = 0; b < nb; o += blk[b].dim, ++b)
        for (int c = 0; c < blk[b].dim; ++c) g += blk[b].R[k * blk[b].dim + c] * r[o + c];
      s += g * g;
    }
    sys->K2[i] = s;
  }

  // fibres of layer j: rows with equal indices outside the layer's columns, keys
  // lexicographic (column order), rows ascending
  for (int layer = 1; layer <= nl; ++layer) {
    const int own = sys->lown[layer - 1], dj = sys->ldim[layer - 1];
    auto key_less = [&](int32_t x, int32_t y) {
      for (int k = 0; k < S; ++k) {
        if (k >= own && k < own + dj) continue;
        const int32_t a = sys->mn[(int64_t)x * S + k], b = sys->mn[(int64_t)y * S + k];
        if (a != b) return a < b;
      }
      return false;
    };
    std::vector<int32_t> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), key_less);
    FibreTable& ft = sys->fib[layer - 1];
    ft.rows = order;
    ft.ptr.clear();
    ft.ptr.push_back(0);
    for (int64_t i = 1; i <= N; ++i)
      if (i == N || key_less(order[i - 1], order[i]) || key_less(order[i], order[i - 1]))
        ft.ptr.push_back((int32_t)i);
    if (N == 0) ft.ptr.assign(1, 0);
    ft.maxL = 0;
    for (size_t f = 0; f + 1 < ft.ptr.size(); ++f) ft.maxL = std::max(ft.maxL, ft.ptr[f + 1] - ft.ptr[f]);
  }

  // neighbour tables of the potential terms: row with the layer's columns shifted by -p,
  // the other columns fixed
  std::unordered_map<uint64_t, int32_t> where;
  where.reserve((size_t)N * 2);
  for (int64_t i = 0; i < N; ++i) where[pack_key(&sys->mn[i * S], S)] = (int32_t)i;
  for (int j = 0; j < nl; ++j) {
    const Stencil& St = sys->pot[j];
    const int own = sys->lown[j], dj = sys->ldim[j];
    sys->nbr[j].assign((size_t)N * St.nv, -1);
    std::vector<int32_t> v(S);
    for (int64_t i = 0; i < N; ++i)
      for (int p = 0; p < St.nv; ++p) {
        for (int k = 0; k < S; ++k) v[k] = sys->mn[i * S + k];
        bool fits = true;
        for (int k = 0; k < dj; ++k) {
          v[own + k] -= St.idx[p * dj + k];
          fits = fits && std::abs(v[own + k]) <= keymax;
        }
        if (!fits) continue;
        auto it = where.find(pack_key(v.data(), S));
        if (it != where.end()) sys->nbr[j][i * St.nv + p] = it->second;
      }
  }
  return LSX_OK;
}

// Layers from lattices (Sec. 2): one block per layer with embedding G_j = 2 pi A_j^{-T};
// the ball cutoff is one group over all blocks, the product cutoff one group per block.
static lsx_status create_system(int32_t d, int32_t nl, const double* const* A, double Ec, int32_t cutoff,
                                const int32_t* nv, const int32_t* const* v_idx, const double* const* v_re,
                                const double* const* v_im, lsx_system** out) {
  if (!out || !A) return fail(LSX_E_INVALID, "null argument");
  if (d != 1 && d != 2) return fail(LSX_E_INVALID, "d must be 1 or 2");
  if (nl < 2 || nl > kMaxLayers) return fail(LSX_E_INVALID, "number of layers must be 2 or 3");
  for (int j = 0; j < nl; ++j)
    if (!A[j]) return fail(LSX_E_INVALID, "null lattice matrix");
  if (!(Ec > 0.0) || !std::isfinite(Ec)) return fail(LSX_E_INVALID, "Ec must be finite and > 0");
  if (cutoff != LSX_CUTOFF_BALL && cutoff != LSX_CUTOFF_PRODUCT) return fail(LSX_E_INVALID, "bad cutoff");
  std::unique_ptr<lsx_system> sys(new (std::nothrow) lsx_system());
  if (!sys) return fail(LSX_E_OOM, "host allocation failed");
  sys->d = d;
  sys->nl = nl;
  sys->standard = true;
  sys->Ec = Ec;
  sys->cutoff = cutoff;
  BlockSpec blk[kMaxLayers];
  int group[kMaxLayers];
  for (int j = 0; j < nl; ++j) {
    for (int k = 0; k < d * d; ++k) sys->A[j][k] = A[j][k];
    if (!reciprocal(d, sys->A[j], sys->B[j]))
      return fail(LSX_E_INVALID, "lattice matrix A" + std::to_string(j + 1) + " is singular or non-finite");
    blk[j].dim = d;
    for (int k = 0; k < d * d; ++k) blk[j].R[k] = sys->B[j][k];
    group[j] = cutoff == LSX_CUTOFF_BALL ? 0 : j;
    sys->lown[j] = j * d;
    sys->ldim[j] = d;
  }
  for (int j = 0; j < nl; ++j)
    LSX_TRY(build_stencil(d, nv ? nv[j] : 0, v_idx ? v_idx[j] : nullptr, v_re ? v_re[j] : nullptr,
                          v_im ? v_im[j] : nullptr, sys->pot[j], j + 1));
  LSX_TRY(build_lifted(sys.get(), d, nl, blk, group, Ec));
  *out = sys.release();
  return LSX_OK;
}

extern "C" lsx_status lsx_system_create_blocks(int32_t D, int32_t nblocks, const int32_t* block_dim,
                                               const double* const* R, const int32_t* group, double Ec,
                                               int32_t nlayers, const int32_t* layer_first,
                                               const int32_t* layer_count, const int32_t* nv,
                                               const int32_t* const* v_idx, const double* const* v_re,
                                               const double* const* v_im, lsx_system** out) {
  if (!out || !block_dim || !R || !group || !layer_first || !layer_count || !nv || !v_idx || !v_re || !v_im)
    return fail(LSX_E_INVALID, "null argument");
  if (D != 1 && D != 2) return fail(LSX_E_INVALID, "physical dimension must be 1 or 2");
  if (nblocks < 1 || nblocks > kMaxBlocks) return fail(LSX_E_INVALID, "number of blocks must be 1 to 4");
  if (nlayers < 2 || nlayers > kMaxLayers) return fail(LSX_E_INVALID, "number of layers must be 2 or 3");
  if (!(Ec > 0.0) || !std::isfinite(Ec)) return fail(LSX_E_INVALID, "Ec must be finite and > 0");
  BlockSpec blk[kMaxBlocks];
  int grp[kMaxBlocks];
  int off[kMaxBlocks + 1] = {0};
  bool used[kMaxBlocks] = {false, false, false, false};
  for (int b = 0; b < nblocks; ++b) {
    if (block_dim[b] != 1 && block_dim[b] != 2) return fail(LSX_E_INVALID, "block dimension must be 1 or 2");
    if (!R[b]) return fail(LSX_E_INVALID, "null block embedding");
    if (group[b] < 0 || group[b] >= nblocks) return fail(LSX_E_INVALID, "cutoff group out of range");
    blk[b].dim = block_dim[b];
    // R[b] column-major D x dim (column c = the wavevector of index component c)
    for (int k = 0; k < D; ++k)
      for (int c = 0; c < block_dim[b]; ++c) {
        const double x = R[b][k + D * c];
        if (!std::isfinite(x)) return fail(LSX_E_INVALID, "non-finite block embedding");
        blk[b].R[k * block_dim[b] + c] = x;
      }
    grp[b] = group[b];
    used[group[b]] = true;
    off[b + 1] = off[b] + block_dim[b];
  }
  for (int g = 0; g < nblocks; ++g)
    if (!used[g] && g < *std::max_element(grp, grp + nblocks))
      return fail(LSX_E_INVALID, "cutoff groups must be numbered 0, 1, ... without gaps");
  if (off[nblocks] > kMaxIndex) return fail(LSX_E_INVALID, "lifted index longer than 6 entries");
  std::unique_ptr<lsx_system> sys(new (std::nothrow) lsx_system());
  if (!sys) return fail(LSX_E_OOM, "host allocation failed");
  sys->d = D;
  sys->nl = nlayers;
  sys->standard = false;
  sys->Ec = Ec;
  sys->cutoff = -1;
  for (int j = 0; j < nlayers; ++j) {
    const int f = layer_first[j], c = layer_count[j];
    if (f < 0 || c < 1 || f + c > nblocks) return fail(LSX_E_INVALID, "layer block range out of range");
    sys->lown[j] = off[f];
    sys->ldim[j] = off[f + c] - off[f];
  }
  // the last layer's fibres (fixed leading columns) must be contiguous runs of the canonical
  // order: its block range has to end with the last block
  if (layer_first[nlayers - 1] + layer_count[nlayers - 1] != nblocks)
    return fail(LSX_E_INVALID, "the last layer must couple the last block");
  for (int j = 0; j < nlayers; ++j)
    LSX_TRY(build_stencil(sys->ldim[j], nv[j], v_idx[j], v_re[j], v_im[j], sys->pot[j], j + 1));
  LSX_TRY(build_lifted(sys.get(), D, nblocks, blk, grp, Ec));
  *out = sys.release();
  return LSX_OK;
}

extern "C" lsx_status lsx_system_create(int32_t d, const double* A1, const double* A2, double Ec, int32_t cutoff,
                                        int32_t nv1, const int32_t* v1_idx, const double* v1_re,
                                        const double* v1_im, int32_t nv2, const int32_t* v2_idx,
                                        const double* v2_re, const double* v2_im, lsx_system** out) {
  if (!A1 || !A2) return fail(LSX_E_INVALID, "null argument");
  const double* A[2] = {A1, A2};
  const int32_t nv[2] = {nv1, nv2};
  const int32_t* idx[2] = {v1_idx, v2_idx};
  const double* re[2] = {v1_re, v2_re};
  const double* im[2] = {v1_im, v2_im};
  return create_system(d, 2, A, Ec, cutoff, nv, idx, re, im, out);
}

extern "C" lsx_status lsx_system_create_layers(int32_t d, int32_t nlayers, const double* const* A, double Ec,
                                               int32_t cutoff, const int32_t* nv, const int32_t* const* v_idx,
                                               const double* const* v_re, const double* const* v_im,
                                               lsx_system** out) {
  if (!nv || !v_idx || !v_re || !v_im) return fail(LSX_E_INVALID, "null potential arrays");
  return create_system(d, nlayers, A, Ec, cutoff, nv, v_idx, v_re, v_im, out);
}

extern "C" lsx_status lsx_system_layers(const lsx_system* sys, int32_t* nlayers, int64_t* nfibres) {
  if (!sys) return fail(LSX_E_INVALID, "null system");
  if (nlayers) *nlayers = sys->nl;
  if (nfibres)
    for (int j = 0; j < sys->nl; ++j) nfibres[j] = (int64_t)sys->fib[j].ptr.size() - 1;
  return LSX_OK;
}

extern "C" lsx_status lsx_system_size(const lsx_system* sys, int64_t* N, int64_t* nf1, int64_t* nf2) {
  if (!sys) return fail(LSX_E_INVALID, "null system");
  if (N) *N = sys->N;
  if (nf1) *nf1 = (int64_t)sys->fib[0].ptr.size() - 1;
  if (nf2) *nf2 = (int64_t)sys->fib[1].ptr.size() - 1;
  return LSX_OK;
}

extern "C" lsx_status lsx_index_get(const lsx_system* sys, int32_t* mn) {
  if (!sys || !mn) return fail(LSX_E_INVALID, "null argument");
  if (!sys->mn.empty()) std::memcpy(mn, sys->mn.data(), sys->mn.size() * sizeof(int32_t));
  return LSX_OK;
}

extern "C" lsx_status lsx_fibre_get(const lsx_system* sys, int32_t layer, int32_t* ptr, int32_t* rows) {
  if (!sys) return fail(LSX_E_INVALID, "null system");
  if (layer < 1 || layer > sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  const FibreTable& ft = sys->fib[layer - 1];
  if (ptr) std::memcpy(ptr, ft.ptr.data(), ft.ptr.size() * sizeof(int32_t));
  if (rows && !ft.rows.empty()) std::memcpy(rows, ft.rows.data(), ft.rows.size() * sizeof(int32_t));
  return LSX_OK;
}

extern "C" lsx_status lsx_system_create_desc(const lsx_system_desc* desc, lsx_system** out) {
  if (!desc) return fail(LSX_E_INVALID, "null descriptor");
  return lsx_system_create(desc->d, desc->A1, desc->A2, desc->Ec, desc->cutoff, desc->nv[0], desc->v_idx[0],
                           desc->v_re[0], desc->v_im[0], desc->nv[1], desc->v_idx[1], desc->v_re[1],
                           desc->v_im[1], out);
}

extern "C" lsx_status lsx_index_size(const lsx_system* sys, int64_t* N) {
  if (!sys || !N) return fail(LSX_E_INVALID, "null argument");
  *N = sys->N;
  return LSX_OK;
}

extern "C" lsx_status lsx_fibre_info(const lsx_system* sys, int32_t layer, int64_t* nfibres, int32_t* lengths) {
  if (!sys) return fail(LSX_E_INVALID, "null system");
  if (layer < 1 || layer > sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  const FibreTable& ft = sys->fib[layer - 1];
  const int64_t nf = (int64_t)ft.ptr.size() - 1;
  if (nfibres) *nfibres = nf;
  if (lengths)
    for (int64_t f = 0; f < nf; ++f) lengths[f] = ft.ptr[f + 1] - ft.ptr[f];
  return LSX_OK;
}

extern "C" lsx_status lsx_system_destroy(lsx_system* sys) {
  if (!sys) return LSX_OK;
  if (sys->nplans > 0) return fail(LSX_E_STATE, "system still has live plans");
  delete sys;
  return LSX_OK;
}

// ================================================================ plan
struct PropSet {
  bool present = false;
  double t = 0.0;
  DBuf<char> data;
  std::vector<int64_t> h_off;
  DBuf<int64_t> off;
};

struct LayerDev {
  int nf = 0;
  int maxL = 0;
  std::vector<int32_t> h_ptr;
  std::vector<int64_t> h_poff;  // byte offset of each fibre's propagator (same for every t)
  std::vector<int32_t> h_d0;    // fibre position of each fibre's diagonal (its representative's)
  std::vector<int32_t> rep;     // distinct-propagator slot of each fibre
  int nunique = 0;
  // The plan's order of the layer's rows (fibre position -> canonical index): the system's
  // fibres with their rows ascending, except that a fibre sharing its representative's
  // propagator through a point symmetry lists the images of the representative's rows.
  std::vector<int32_t> h_rows;
  std::vector<int32_t> sym_rep;  // representative fibre under the point symmetries (empty: none)
  bool ident = false;            // h_rows is the identity (the canonical order)
  DBuf<int32_t> ptr, rows;
  DBuf<int32_t> nbr;
  DBuf<double2> v;  // stencil values (for the energy)
  PropSet prop[3];  // sub-step slots, times per scheme in scheme_times()
  // Band of every 16-row block of every stored propagator, as fibre positions [lo, hi): row
  // block rb of distinct propagator b is entry h_boff[b] + rb; the union over the layer's slots.
  std::vector<int64_t> h_boff;
  std::vector<int32_t> band_lo, band_hi;
  DBuf<int32_t> d_band;  // the same bands on the device, (lo, hi) pairs (empty: dense products)
  // Fibres that share a stored propagator, in groups of up to kOrbitMax in fibre order (a
  // fibre without partners is a group of one), and the device table of the groups for the
  // single-state orbit passes (PassArgs::orbit; empty when no fibre shares); orbit_max: the
  // largest group
  std::vector<std::vector<int>> groups;
  DBuf<int32_t> d_orbit;
  int orbit_max = 0;
};

// Band of row blocks [rb0, rb0 + n) of fibre f (those inside the fibre) as fibre positions
// [k0, k1): the union of the blocks' bands.
static void fibre_band(const LayerDev& ld, int f, int rb0, int n, int32_t& k0, int32_t& k1) {
  const int L = ld.h_ptr[f + 1] - ld.h_ptr[f];
  const int nrb = (L + 15) / 16;
  k0 = kBandEnd;
  k1 = 0;
  if (!ld.h_boff.empty()) {
    const int64_t base = ld.h_boff[ld.rep[f]];
    for (int rb = rb0; rb < std::min(nrb, rb0 + n); ++rb) {
      k0 = std::min(k0, ld.band_lo[base + rb]);
      k1 = std::max(k1, ld.band_hi[base + rb]);
    }
  }
  if (k1 <= k0) {
    k0 = 0;
    k1 = kBandEnd;
  }
}

struct lsx_plan {
  lsx_system* sys = nullptr;
  double tau = 0.0, kappa = 0.0;
  // propagator entries with |Re| + |Im| below band_tol are left out of the products, at the
  // granularity of the storage's column chunks (0: every chunk is multiplied)
  double band_tol = 0.0;
  int scheme = LSX_STRANG, precision = LSX_FP64, fmt = PF_F64;
  DBuf<double> K2;
  DBuf<double2> diag;  // mixed formats: per fibre-row diagonal, [layer*3+slot] blocks of N
  DBuf<double2> phase[3];  // exp(-i kappa t |K|^2/2) for the scheme's phase times
  // pos[j]: position of canonical index i in the layer-(j+1) fibre order; xmap[j][k]:
  // layer-(j+1) fibre position -> layer-(k+1) fibre position.  Held for the layers whose order
  // is not the canonical one (every layer but the last, and the last too when point symmetries
  // reorder its fibres).
  DBuf<int32_t> pos[kMaxLayers];
  DBuf<int32_t> xmap[kMaxLayers][kMaxLayers];
  DBuf<int32_t> iota;  // identity table (batched gathers over systems whose table is the identity)
  int nsym = 0;        // point symmetries the propagators are shared over (identity excluded)
  DBuf<double2> zero;  // 1 KiB of zeros (out-of-range operand loads of the passes)
  LayerDev L[kMaxLayers];
  int nstates = 0;
  int max_w = 0;  // states with more wavepackets are refused (0: no limit)
};

// Index table of layer `layer`'s fibre positions inside an array of layout `layout` (layout 0:
// canonical order; layout j: layer-j fibre order); nullptr when the two coincide.  Without
// point-symmetry sharing the last layer's fibres are contiguous runs of the canonical order,
// so layouts 0 and nl coincide.
static const int32_t* layout_map(const lsx_plan* pl, int layer, int layout) {
  if (layout == layer) return nullptr;
  const LayerDev& ld = pl->L[layer - 1];
  if (layout == 0) return ld.ident ? nullptr : ld.rows.p;  // fibre position -> canonical index
  if (pl->L[layout - 1].ident) return ld.rows.p;             // that layout is the canonical order
  if (ld.ident) return pl->pos[layout - 1].p;                // canonical index -> fibre position
  return pl->xmap[layer - 1][layout - 1].p;
}

// Sub-step flow of a scheme: 0 exact exponential, 1 backward Euler, 2 Crank-Nicolson.
static int scheme_flow(int scheme) { return scheme == LSX_LIE_BE ? 1 : (scheme == LSX_STRANG_CN ? 2 : 0); }
static bool scheme_strang(int scheme) { return scheme == LSX_STRANG || scheme == LSX_STRANG_CN; }

// Yoshida's symmetric triple jump S4(tau) = S2(g1 tau) S2(g0 tau) S2(g1 tau) of Strang steps
// S2, with 2 g1 + g0 = 1 and 2 g1^3 + g0^3 = 0 (fourth order).
static const double kYoshidaG1 = 1.0 / (2.0 - std::cbrt(2.0));
static const double kYoshidaG0 = 1.0 - 2.0 * kYoshidaG1;

// Times of a scheme's propagator slots per layer and of its kinetic-phase tables (NaN: the
// slot is not used).
//  Lie, BE-Lie        : layer 1 {tau}, layer 2 {tau}, phase {tau}
//  Strang, CN-Strang  : layer 1 {tau, tau/2}, layer 2 {tau}, phase {tau, tau/2}
//  Yoshida (4th order): layer 1 {g1 tau, g1 tau/2, (g1+g0) tau/2}, layer 2 {g1 tau, -, g0 tau},
//                       phase {g1 tau/2, g0 tau/2}
// Three layers:
//  Lie, BE-Lie        : every layer {tau}, phase {tau}
//  Strang, CN-Strang  : layer 1 {tau, tau/2}, layer 2 {-, tau/2}, layer 3 {tau}, phase {tau, tau/2}
//  Yoshida            : layer 1 {g1 tau, g1 tau/2, (g1+g0) tau/2}, layer 2 {g1 tau/2, g0 tau/2},
//                       layer 3 {g1 tau, -, g0 tau}, phase {g1 tau/2, g0 tau/2}
struct SchemeTimes {
  double t[kMaxLayers][3];
  double ph[3];
};
static SchemeTimes scheme_times(int scheme, double tau, int nl) {
  const double X = std::nan("");
  if (nl == 3) {
    if (scheme == LSX_YOSHIDA4) {
      const double g1 = kYoshidaG1, g0 = kYoshidaG0;
      return {{{g1 * tau, 0.5 * g1 * tau, 0.5 * (g1 + g0) * tau},
               {0.5 * g1 * tau, 0.5 * g0 * tau, X},
               {g1 * tau, X, g0 * tau}},
              {0.5 * g1 * tau, 0.5 * g0 * tau, X}};
    }
    if (scheme_strang(scheme)) return {{{tau, 0.5 * tau, X}, {X, 0.5 * tau, X}, {tau, X, X}}, {tau, 0.5 * tau, X}};
    return {{{tau, X, X}, {tau, X, X}, {tau, X, X}}, {tau, X, X}};
  }
  if (scheme == LSX_YOSHIDA4) {
    const double g1 = kYoshidaG1, g0 = kYoshidaG0;
    return {{{g1 * tau, 0.5 * g1 * tau, 0.5 * (g1 + g0) * tau}, {g1 * tau, X, g0 * tau}, {X, X, X}},
            {0.5 * g1 * tau, 0.5 * g0 * tau, X}};
  }
  if (scheme_strang(scheme)) return {{{tau, 0.5 * tau, X}, {tau, X, X}, {X, X, X}}, {tau, 0.5 * tau, X}};
  return {{{tau, X, X}, {tau, X, X}, {X, X, X}}, {tau, X, X}};
}

// ---------------------------------------------------------------- point symmetries
// A rotation R of the plane (in 1D, x -> -x) is a symmetry of a lattice-built system when, for
// every layer j, it maps the reciprocal lattice onto itself, R B_j = B_j M_j with M_j an integer
// matrix, keeps the layer's potential (its coefficient at M_j m equals the one at m) and maps
// the lifted index set onto itself (the cutoff depends on |G_j m_j| only).  The lifted
// wavevector K = sum_j B_j m_j then goes to R K, |K|^2 is unchanged, and the fibre Hamiltonian
// H_j (eq. 3.6, with its kinetic share) at the fibre whose fixed indices are (M_k m_k)_{k != j}
// is the one at (m_k)_{k != j} with every row (m_j, ...) relabelled (M_j m_j, ...).  So the
// fibres of an orbit have permuted copies of one Hamiltonian, and every function of it (exact
// flow, backward Euler or Crank-Nicolson factor) is the same permuted copy.  Ordering each
// fibre's rows as the images of its representative's rows makes the stored propagators equal.
struct PointSym {
  int32_t M[kMaxLayers][4];  // d x d integer matrix per layer, row-major
};

static std::vector<PointSym> find_point_symmetries(const lsx_system* sys) {
  std::vector<PointSym> out;
  if (!sys->standard || sys->N == 0) return out;
  const int d = sys->d, nl = sys->nl;
  std::vector<std::vector<double>> Rs;
  if (d == 1) {
    Rs.push_back({-1.0});
  } else {
    for (int k = 1; k < 12; ++k) {
      const double th = 2.0 * M_PI * k / 12.0;
      Rs.push_back({std::cos(th), -std::sin(th), std::sin(th), std::cos(th)});
    }
  }
  std::unordered_map<uint64_t, int32_t> where;
  const int S = sys->S;
  for (const auto& R : Rs) {
    PointSym g{};
    bool ok = true;
    for (int j = 0; j < nl && ok; ++j) {
      // M = B^{-1} R B with B row-major (columns: reciprocal primitive vectors)
      const double* B = sys->B[j];
      double Bi[4];
      if (d == 1) {
        Bi[0] = 1.0 / B[0];
      } else {
        const double det = B[0] * B[3] - B[1] * B[2];
        Bi[0] = B[3] / det;
        Bi[1] = -B[1] / det;
        Bi[2] = -B[2] / det;
        Bi[3] = B[0] / det;
      }
      for (int r = 0; r < d && ok; ++r)
        for (int c = 0; c < d && ok; ++c) {
          double x = 0.0;
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) x += Bi[r * d + a] * R[a * d + b] * B[b * d + c];
          const double xr = std::nearbyint(x);
          if (std::fabs(x - xr) > 1e-9) ok = false;
          g.M[j][r * d + c] = (int32_t)xr;
        }
      // the potential's coefficients are permuted among themselves with equal values
      const Stencil& st = sys->pot[j];
      double vmax = 0.0;
      for (int e = 0; e < st.nv; ++e) vmax = std::max(vmax, std::hypot(st.re[e], st.im[e]));
      for (int e = 0; e < st.nv && ok; ++e) {
        int32_t im[2];
        for (int r = 0; r < d; ++r) {
          int64_t acc = 0;
          for (int c = 0; c < d; ++c) acc += (int64_t)g.M[j][r * d + c] * st.idx[(size_t)e * d + c];
          im[r] = (int32_t)acc;
        }
        int f = -1;
        for (int e2 = 0; e2 < st.nv && f < 0; ++e2) {
          bool same = true;
          for (int r = 0; r < d; ++r) same = same && st.idx[(size_t)e2 * d + r] == im[r];
          if (same) f = e2;
        }
        if (f < 0 || std::fabs(st.re[f] - st.re[e]) > 1e-14 * vmax || std::fabs(st.im[f] - st.im[e]) > 1e-14 * vmax)
          ok = false;
      }
    }
    if (!ok) continue;
    // the lifted index set maps onto itself
    if (where.empty())
      for (int64_t i = 0; i < sys->N; ++i) where[pack_key(&sys->mn[i * S], S)] = (int32_t)i;
    int32_t img[kMaxIndex];
    for (int64_t i = 0; i < sys->N && ok; ++i) {
      const int32_t* m = &sys->mn[i * S];
      for (int j = 0; j < nl; ++j)
        for (int r = 0; r < d; ++r) {
          int64_t acc = 0;
          for (int c = 0; c < d; ++c) acc += (int64_t)g.M[j][r * d + c] * m[j * d + c];
          if (std::llabs(acc) > (S <= 4 ? 32767 : 511)) ok = false;
          img[j * d + r] = (int32_t)acc;
        }
      ok = ok && where.count(pack_key(img, S)) > 0;
    }
    if (ok) out.push_back(g);
  }
  return out;
}

extern "C" lsx_status lsx_system_symmetries(const lsx_system* sys, int32_t* nsym, int32_t* M) {
  if (!sys || !nsym) return fail(LSX_E_INVALID, "null argument");
  const std::vector<PointSym> g = find_point_symmetries(sys);
  *nsym = (int32_t)g.size();
  if (M) {
    const int d = sys->d, nl = sys->nl;
    for (size_t e = 0; e < g.size(); ++e)
      for (int j = 0; j < nl; ++j)
        for (int k = 0; k < d * d; ++k) M[(e * nl + j) * d * d + k] = g[e].M[j][k];
  }
  return LSX_OK;
}

// The plan's row order of every layer and, with point symmetries, each fibre's representative.
static void plan_orders(lsx_plan* pl, bool use_sym) {
  const lsx_system* sys = pl->sys;
  const int nl = sys->nl, d = sys->d, S = sys->S;
  std::vector<PointSym> syms;
  if (use_sym) syms = find_point_symmetries(sys);
  pl->nsym = (int)syms.size();
  std::unordered_map<uint64_t, int32_t> where;
  if (!syms.empty())
    for (int64_t i = 0; i < sys->N; ++i) where[pack_key(&sys->mn[i * S], S)] = (int32_t)i;
  for (int j = 0; j < nl; ++j) {
    LayerDev& ld = pl->L[j];
    const FibreTable& ft = sys->fib[j];
    const int nf = (int)ft.ptr.size() - 1;
    ld.h_rows = ft.rows;
    ld.sym_rep.clear();
    if (!syms.empty()) {
      // fibre of every canonical row
      std::vector<int32_t> fib((size_t)sys->N);
      for (int f = 0; f < nf; ++f)
        for (int a = ft.ptr[f]; a < ft.ptr[f + 1]; ++a) fib[ft.rows[a]] = f;
      ld.sym_rep.assign(nf, -1);
      int32_t img[kMaxIndex];
      for (int f = 0; f < nf; ++f) {
        if (ld.sym_rep[f] >= 0) continue;
        ld.sym_rep[f] = f;
        const int r0 = ft.ptr[f], L = ft.ptr[f + 1] - r0;
        for (const PointSym& g : syms) {
          // image of the fibre's first row decides the image fibre
          auto image = [&](int32_t row) {
            const int32_t* m = &sys->mn[(size_t)row * S];
            for (int k = 0; k < nl; ++k)
              for (int r = 0; r < d; ++r) {
                int64_t acc = 0;
                for (int c = 0; c < d; ++c) acc += (int64_t)g.M[k][r * d + c] * m[k * d + c];
                img[k * d + r] = (int32_t)acc;
              }
            return where.at(pack_key(img, S));
          };
          const int f2 = fib[image(ft.rows[r0])];
          if (ld.sym_rep[f2] >= 0) continue;
          if (ft.ptr[f2 + 1] - ft.ptr[f2] != L) continue;  // cannot happen for a symmetry
          bool same_fibre = true;
          std::vector<int32_t> rows(L);
          for (int a = 0; a < L; ++a) {
            rows[a] = image(ft.rows[r0 + a]);
            same_fibre = same_fibre && fib[rows[a]] == f2;
          }
          if (!same_fibre) continue;
          ld.sym_rep[f2] = f;
          std::copy(rows.begin(), rows.end(), ld.h_rows.begin() + ft.ptr[f2]);
        }
      }
    }
    ld.ident = true;
    for (int64_t p = 0; p < sys->N && ld.ident; ++p) ld.ident = ld.h_rows[p] == (int32_t)p;
  }
}

// Fibres longer than this many rows (after the complex embedding) take the blocked solver.
static constexpr int kBlockedMin = 96;

// Blocked two-sided Jacobi (see lsx_kernels.hip) of the matrices `sel` of a precompute batch:
// sweeps of round-robin block rounds until a sweep rotates nothing, at most maxsweeps; the
// matrices that converge drop out after each sweep.  info[m] receives the sweeps of matrix m,
// or -1 without convergence.
static lsx_status block_jacobi(hipStream_t s, const std::vector<int32_t>& sel, const std::vector<int32_t>& ndim,
                               double* A, double* VT, const int64_t* d_moff, const int32_t* d_ndim, double* lam,
                               const int64_t* d_loff, int maxsweeps, std::vector<int32_t>& info) {
  const int nm = (int)ndim.size();
  std::vector<int32_t> act(sel);
  std::stable_sort(act.begin(), act.end(), [&](int x, int y) { return ndim[x] > ndim[y]; });
  int64_t qsize = 0;
  for (int m : act) qsize += (int64_t)(ndim[m] / 32) * 1024;
  DBuf<int32_t> d_sel, d_mat, d_pp, d_pt, d_flag;
  DBuf<double> d_tiny, d_Q;
  LSX_TRY(d_sel.upload(sel, s));
  LSX_TRY(d_tiny.alloc(nm));
  LSX_TRY(d_flag.alloc(nm));
  LSX_TRY(d_Q.alloc(qsize));
  BJArgs g;
  g.A = A;
  g.VT = VT;
  g.moff = d_moff;
  g.ndim = d_ndim;
  g.tiny = d_tiny.p;
  g.Q = d_Q.p;
  g.flag = d_flag.p;
  LSX_HIP_TRY(launch_bj_init(s, (int)sel.size(), d_sel.p, g));
  std::vector<int32_t> flag(nm, 0);
  int sweep = 0;
  for (; sweep < maxsweeps && !act.empty(); ++sweep) {
    const int na = (int)act.size();
    std::vector<int32_t> pp(na + 1, 0), pt(na + 1, 0);
    for (int a = 0; a < na; ++a) {
      const int np = ndim[act[a]] / 32;
      pp[a + 1] = pp[a] + np;
      pt[a + 1] = pt[a] + 2 * np * np;
    }
    LSX_TRY(d_mat.upload(act, s));
    LSX_TRY(d_pp.upload(pp, s));
    LSX_TRY(d_pt.upload(pt, s));
    LSX_HIP_TRY(hipMemsetAsync(d_flag.p, 0, nm * sizeof(int32_t), s));
    g.mat = d_mat.p;
    g.pfx_pairs = d_pp.p;
    g.pfx_tiles = d_pt.p;
    const int rounds = ndim[act[0]] / 16 - 1;
    int count = na;
    for (int r = 0; r < rounds; ++r) {
      // matrices with more than r + 1 blocks take part (a prefix: act is sorted by size)
      while (count > 0 && ndim[act[count - 1]] / 16 - 1 <= r) --count;
      g.count = count;
      g.round = r;
      LSX_HIP_TRY(launch_bj_round(s, pp[count], pt[count], g));
    }
    LSX_HIP_TRY(hipMemcpyAsync(flag.data(), d_flag.p, nm * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSX_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> keep;
    for (int m : act) {
      if (flag[m]) keep.push_back(m);
      else info[m] = sweep + 1;
    }
    act.swap(keep);
  }
  for (int m : act) info[m] = -1;
  LSX_HIP_TRY(launch_bj_finish(s, (int)sel.size(), d_sel.p, g, lam, d_loff));
  LSX_HIP_TRY(hipStreamSynchronize(s));
  return LSX_OK;
}

static lsx_status precompute_layer(lsx_plan* pl, int layer, hipStream_t s) {
  lsx_system* sys = pl->sys;
  LayerDev& ld = pl->L[layer - 1];
  const FibreTable& ft = sys->fib[layer - 1];
  const Stencil& S = sys->pot[layer - 1];
  const int nf = ld.nf;
  if (nf == 0) return LSX_OK;
  const int d = sys->ldim[layer - 1];  // entries of the index the layer's potential couples
  const int stride = sys->S;
  const int own = sys->lown[layer - 1];
  // With kappa = 1 a fibre Hamiltonian is the potential restricted to the fibre's window
  // of own indices, which is translation invariant: fibres whose windows coincide up to a
  // shift share one eigendecomposition and one stored propagator.
  ld.rep.resize(nf);
  std::vector<int32_t> uniq;
  if (pl->kappa == 1.0) {
    std::map<std::vector<int32_t>, int> seen;
    for (int f = 0; f < nf; ++f) {
      std::vector<int32_t> key;
      const int r0 = ft.ptr[f], L = ft.ptr[f + 1] - r0;
      key.reserve((size_t)L * d);
      const int32_t* base = &sys->mn[(int64_t)ft.rows[r0] * stride + own];
      for (int a = 0; a < L; ++a)
        for (int k = 0; k < d; ++k) key.push_back(sys->mn[(int64_t)ft.rows[r0 + a] * stride + own + k] - base[k]);
      auto it = seen.find(key);
      if (it == seen.end()) {
        seen.emplace(std::move(key), (int)uniq.size());
        ld.rep[f] = (int)uniq.size();
        uniq.push_back(f);
      } else {
        ld.rep[f] = it->second;
      }
    }
  } else if (!ld.sym_rep.empty()) {
    // fibres of one point-symmetry orbit share their representative's propagator
    std::vector<int32_t> slot(nf, -1);
    for (int f = 0; f < nf; ++f) {
      const int r = ld.sym_rep[f];
      if (slot[r] < 0) {
        slot[r] = (int)uniq.size();
        uniq.push_back(r);
      }
      ld.rep[f] = slot[r];
    }
  } else {
    for (int f = 0; f < nf; ++f) {
      ld.rep[f] = f;
      uniq.push_back(f);
    }
  }
  const int nu = (int)uniq.size();
  ld.nunique = nu;
  const int embed = S.real ? 0 : 1;
  std::vector<int32_t> ndim(nu), emb(nu, embed);
  std::vector<int64_t> moff(nu), loff(nu);
  int64_t mt = 0, lt = 0;
  int maxn = 0, maxL = 0;
  // Matrices of more than kBlockedMin rows take the blocked solver (padded to a multiple of 32),
  // the others the scalar one (padded to even); LSX_BLOCKED_JACOBI=0 keeps every fibre scalar.
  const int blocked_min = env_int("LSX_BLOCKED_JACOBI", 1) != 0 ? kBlockedMin : 1 << 30;
  std::vector<int32_t> sel_s, sel_b;
  int maxn_s = 0;
  for (int b = 0; b < nu; ++b) {
    const int f = uniq[b];
    const int L = ft.ptr[f + 1] - ft.ptr[f];
    maxL = std::max(maxL, L);
    int n = embed ? 2 * L : L;
    if (n > blocked_min) {
      n = round_up(n, 32);
      sel_b.push_back(b);
    } else {
      n += (n & 1);
      if (n < 2) n = 2;
      sel_s.push_back(b);
      maxn_s = std::max(maxn_s, n);
    }
    ndim[b] = n;
    maxn = std::max(maxn, n);
    moff[b] = mt;
    loff[b] = lt;
    mt += (int64_t)n * n;
    lt += n;
  }
  if (maxn > 8192) return fail(LSX_E_INVALID, "fibre too long for the eigensolver (max 8192)");
  DBuf<int32_t> d_ndim, d_emb, d_info, d_mn, d_vidx, d_fid;
  DBuf<int64_t> d_moff, d_loff;
  DBuf<double> A, VT, lam, d_vre, d_vim;
  DBuf<double2> gh;
  LSX_TRY(d_fid.upload(uniq, s));
  LSX_TRY(d_ndim.upload(ndim, s));
  LSX_TRY(d_emb.upload(emb, s));
  LSX_TRY(d_moff.upload(moff, s));
  LSX_TRY(d_loff.upload(loff, s));
  LSX_TRY(d_mn.upload(sys->mn, s));
  LSX_TRY(d_vidx.upload(S.idx, s));
  LSX_TRY(d_vre.upload(S.re, s));
  LSX_TRY(d_vim.upload(S.im, s));
  LSX_TRY(A.alloc(mt));
  LSX_TRY(VT.alloc(mt));
  LSX_TRY(lam.alloc(lt));
  LSX_TRY(gh.alloc(lt));
  LSX_TRY(d_info.alloc(nu));
  // kinetic share of H_j: (1 - kappa)/nl * |K|^2/2
  const double kfac = (1.0 - pl->kappa) / sys->nl * 0.5;
  LSX_HIP_TRY(launch_assemble(s, nu, d_fid.p, ld.ptr.p, ld.rows.p, d_mn.p, d, stride, own, kfac, pl->K2.p, S.nv,
                              d_vidx.p, d_vre.p, d_vim.p, embed, A.p, d_moff.p, d_ndim.p));
  std::vector<int32_t> info(nu, 0);
  if (!sel_s.empty()) {
    DBuf<int32_t> d_sel;
    LSX_TRY(d_sel.upload(sel_s, s));
    LSX_HIP_TRY(launch_jacobi(s, (int)sel_s.size(), maxn_s, A.p, VT.p, d_moff.p, d_ndim.p, lam.p, d_loff.p,
                              d_info.p, 60, d_sel.p));
    LSX_HIP_TRY(hipMemcpyAsync(info.data(), d_info.p, nu * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSX_HIP_TRY(hipStreamSynchronize(s));
  }
  if (!sel_b.empty())
    LSX_TRY(block_jacobi(s, sel_b, ndim, A.p, VT.p, d_moff.p, d_ndim.p, lam.p, d_loff.p, 60, info));
  if (const char* fe = std::getenv("LSX_TEST_FAIL_EIG"))
    if (std::atoi(fe) == 1) info[0] = -1;
  for (int b = 0; b < nu; ++b)
    if (info[b] < 0)
      return fail(LSX_E_EIG, "Jacobi did not converge for layer " + std::to_string(layer) + " fibre " +
                                 std::to_string(uniq[b]));
  // propagator storage: one slot per distinct fibre; fibres map to their representative
  std::vector<int64_t> uoff(nu);
  int64_t bytes = 0;
  for (int b = 0; b < nu; ++b) {
    uoff[b] = bytes;
    bytes += prop_bytes(pl->fmt, ft.ptr[uniq[b] + 1] - ft.ptr[uniq[b]]);
    bytes = (bytes + 255) & ~(int64_t)255;
  }
  ld.h_poff.resize(nf);
  ld.h_d0.resize(nf);
  for (int f = 0; f < nf; ++f) {
    ld.h_poff[f] = uoff[ld.rep[f]];
    ld.h_d0[f] = ft.ptr[uniq[ld.rep[f]]];
  }
  {
    ld.groups.clear();
    ld.orbit_max = 0;
    std::vector<int> open(nu, -1);  // propagator slot -> its group being filled
    for (int f = 0; f < nf; ++f) {
      int& g = open[ld.rep[f]];
      if (g < 0 || (int)ld.groups[g].size() >= kOrbitMax) {
        g = (int)ld.groups.size();
        ld.groups.emplace_back();
      }
      ld.groups[g].push_back(f);
    }
    for (const std::vector<int>& g : ld.groups) ld.orbit_max = std::max(ld.orbit_max, (int)g.size());
    ld.d_orbit.release();
    if (ld.orbit_max > 1) {
      std::vector<int32_t> tab((size_t)kOrbitStride * ld.groups.size());
      for (size_t g = 0; g < ld.groups.size(); ++g) {
        const std::vector<int>& mem = ld.groups[g];
        tab[g * kOrbitStride] = (int32_t)mem.size();
        for (int m = 0; m < kOrbitMax; ++m) tab[g * kOrbitStride + 1 + m] = ft.ptr[mem[m < (int)mem.size() ? m : 0]];
      }
      LSX_TRY(ld.d_orbit.upload(tab, s));
    }
  }
  // bands of the stored propagators, one entry per 16-row block, united over the slots
  std::vector<int64_t> boff(nu + 1, 0);
  for (int b = 0; b < nu; ++b) boff[b + 1] = boff[b] + (ft.ptr[uniq[b] + 1] - ft.ptr[uniq[b]] + 15) / 16;
  const int64_t nband = boff[nu];
  ld.h_boff = boff;
  const bool banded = pl->band_tol > 0.0;
  const int cw = band_chunk(pl->fmt);
  ld.band_lo.assign(nband, banded ? kBandEnd : 0);
  ld.band_hi.assign(nband, banded ? 0 : kBandEnd);
  DBuf<int64_t> d_boff;
  DBuf<int32_t> d_band;
  std::vector<int32_t> hband;
  if (banded) {
    LSX_TRY(d_boff.upload(boff, s));
    LSX_TRY(d_band.alloc((size_t)2 * nband));
    hband.resize((size_t)2 * nband);
  }
  const int flow = scheme_flow(pl->scheme);
  const SchemeTimes times = scheme_times(pl->scheme, pl->tau, sys->nl);
  for (int h = 0; h < 3; ++h) {
    PropSet& ps = ld.prop[h];
    if (std::isnan(times.t[layer - 1][h])) continue;
    ps.t = times.t[layer - 1][h];
    ps.h_off = ld.h_poff;
    LSX_TRY(ps.data.alloc(bytes));
    LSX_TRY(ps.off.upload(uoff, s));
    LSX_HIP_TRY(hipMemsetAsync(ps.data.p, 0, bytes, s));
    LSX_HIP_TRY(launch_eig_fn(s, lt, lam.p, ps.t, flow, gh.p));
    double2* dg = pl->diag.p ? pl->diag.p + (size_t)((layer - 1) * 3 + h) * sys->N : nullptr;
    LSX_HIP_TRY(launch_form(s, pl->fmt, nu, maxL, d_fid.p, ld.ptr.p, VT.p, d_moff.p, d_ndim.p, d_emb.p, gh.p,
                            d_loff.p, ps.data.p, ps.off.p, dg));
    ps.present = true;
    if (banded && nband > 0) {
      LSX_HIP_TRY(launch_band(s, pl->fmt, nu, d_fid.p, ld.ptr.p, ps.data.p, ps.off.p, d_boff.p, pl->band_tol,
                              d_band.p));
      LSX_HIP_TRY(hipMemcpyAsync(hband.data(), d_band.p, hband.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      LSX_HIP_TRY(hipStreamSynchronize(s));
      for (int64_t i = 0; i < nband; ++i) {
        ld.band_lo[i] = std::min(ld.band_lo[i], hband[2 * i] * cw);
        ld.band_hi[i] = std::max(ld.band_hi[i], hband[2 * i + 1] * cw);
      }
    }
  }
  if (banded && nband > 0) {
    for (int64_t i = 0; i < nband; ++i) {
      hband[2 * i] = ld.band_lo[i];
      hband[2 * i + 1] = ld.band_hi[i];
    }
    LSX_TRY(ld.d_band.upload(hband, s));
  }
  LSX_HIP_TRY(hipStreamSynchronize(s));
  return LSX_OK;
}

// band_req: 0 the default tolerance for the precision (LSX_BAND_TOL overrides it), < 0 dense
// products, > 0 that tolerance.
static lsx_status plan_create(lsx_system* sys, double tau, int32_t scheme, double kappa, int32_t precision,
                              double band_req, void* stream, lsx_plan** out) {
  if (!sys || !out) return fail(LSX_E_INVALID, "null argument");
  if (!std::isfinite(tau) || tau == 0.0) return fail(LSX_E_INVALID, "tau must be finite and nonzero");
  if (scheme != LSX_LIE && scheme != LSX_STRANG && scheme != LSX_LIE_BE && scheme != LSX_STRANG_CN &&
      scheme != LSX_YOSHIDA4)
    return fail(LSX_E_INVALID, "bad scheme");
  if (!(kappa >= 0.0 && kappa <= 1.0)) return fail(LSX_E_INVALID, "kappa must be in [0, 1]");
  if (precision != LSX_FP64 && precision != LSX_MIX_FP32 && precision != LSX_MIX_BF16X3)
    return fail(LSX_E_INVALID, "bad precision");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  lsx_plan* pl = new (std::nothrow) lsx_plan();
  if (!pl) return fail(LSX_E_OOM, "host allocation failed");
  pl->sys = sys;
  pl->tau = tau;
  pl->kappa = kappa;
  pl->scheme = scheme;
  pl->precision = precision;
  pl->fmt = precision == LSX_FP64 ? PF_F64 : (precision == LSX_MIX_FP32 ? PF_F32 : PF_BF16X3);
  // Band tolerance: for FP64 the unit roundoff u = 2^-53, so the entries left out change a pass
  // by at most L u relative, the order of the pass's own rounding bound (and of the accuracy of
  // the computed propagator entries); for the mixed paths 2^-44, at most L 2^-44 per pass
  // (about 5e-11 for fibres of 900 rows), far below the FP32 rounding of the entries that are
  // kept.  LSX_BAND_TOL overrides it (0: dense products).
  if (band_req > 0.0)
    pl->band_tol = band_req;
  else if (band_req == 0.0)
    pl->band_tol = env_double("LSX_BAND_TOL", pl->fmt == PF_F64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -44));
  if (!(pl->band_tol >= 0.0)) pl->band_tol = 0.0;
  auto cleanup = [&](lsx_status st) {
    delete pl;
    return st;
  };
  lsx_status st = pl->K2.upload(sys->K2, s);
  if (st != LSX_OK) return cleanup(st);
  if (pl->fmt != PF_F64) {
    st = pl->diag.alloc((size_t)3 * sys->nl * std::max<int64_t>(sys->N, 1));
    if (st != LSX_OK) return cleanup(st);
  }
  const int nl = sys->nl;
  // window sharing (kappa = 1) and point-symmetry sharing are alternatives: at kappa = 1 the
  // translation-invariant windows already share more; LSX_SYMMETRY=0 turns the latter off
  plan_orders(pl, kappa != 1.0 && env_int("LSX_SYMMETRY", 1) != 0);
  for (int j = 0; j < nl; ++j) {
    LayerDev& ld = pl->L[j];
    const FibreTable& ft = sys->fib[j];
    ld.nf = (int)ft.ptr.size() - 1;
    ld.maxL = ft.maxL;
    ld.h_ptr = ft.ptr;
    if ((st = ld.ptr.upload(ft.ptr, s)) != LSX_OK) return cleanup(st);
    if ((st = ld.rows.upload(ld.h_rows, s)) != LSX_OK) return cleanup(st);
    if ((st = ld.nbr.upload(sys->nbr[j], s)) != LSX_OK) return cleanup(st);
    std::vector<double2> v(sys->pot[j].nv);
    for (int p = 0; p < sys->pot[j].nv; ++p) v[p] = make_double2(sys->pot[j].re[p], sys->pot[j].im[p]);
    if ((st = ld.v.upload(v, s)) != LSX_OK) return cleanup(st);
  }
  {
    // position tables between the layers' orders and the canonical order; a layer whose order
    // is the canonical one (the last layer, unless point symmetries reorder it) needs none
    const size_t n1 = (size_t)std::max<int64_t>(sys->N, 1);
    std::vector<std::vector<int32_t>> pos(nl);
    for (int j = 0; j < nl; ++j) {
      if (pl->L[j].ident) continue;
      pos[j].assign(n1, 0);
      for (int64_t p = 0; p < sys->N; ++p) pos[j][pl->L[j].h_rows[p]] = (int32_t)p;
      if ((st = pl->pos[j].upload(pos[j], s)) != LSX_OK) return cleanup(st);
    }
    for (int j = 0; j < nl; ++j)
      for (int k = 0; k < nl; ++k) {
        if (j == k || pl->L[j].ident || pl->L[k].ident) continue;
        std::vector<int32_t> x(n1, 0);
        for (int64_t p = 0; p < sys->N; ++p) x[p] = pos[k][pl->L[j].h_rows[p]];
        if ((st = pl->xmap[j][k].upload(x, s)) != LSX_OK) return cleanup(st);
      }
    if ((st = pl->zero.upload(std::vector<double2>(64, make_double2(0.0, 0.0)), s)) != LSX_OK) return cleanup(st);
  }
  if (kappa != 0.0) {
    const SchemeTimes times = scheme_times(scheme, tau, nl);
    for (int h = 0; h < 3; ++h) {
      const double t = times.ph[h];
      if (std::isnan(t)) continue;
      if ((st = pl->phase[h].alloc(std::max<int64_t>(sys->N, 1))) != LSX_OK) return cleanup(st);
      if (sys->N > 0) {
        hipError_t e = launch_phase_table(s, sys->N, pl->K2.p, 0.5 * kappa * t, pl->phase[h].p);
        if (e != hipSuccess) return cleanup(fail(LSX_E_HIP, std::string("phase table: ") + hipGetErrorString(e)));
      }
    }
  }
  for (int layer = 1; layer <= nl; ++layer)
    if ((st = precompute_layer(pl, layer, s)) != LSX_OK) return cleanup(st);
  sys->nplans++;
  *out = pl;
  return LSX_OK;
}

extern "C" lsx_status lsx_plan_create(lsx_system* sys, double tau, int32_t scheme, double kappa,
                                      int32_t precision, void* stream, lsx_plan** out) {
  return plan_create(sys, tau, scheme, kappa, precision, 0.0, stream, out);
}

extern "C" lsx_status lsx_plan_create_desc(lsx_system* sys, const lsx_plan_desc* desc, void* stream,
                                           lsx_plan** out) {
  if (!desc) return fail(LSX_E_INVALID, "null descriptor");
  if (desc->max_wavepackets < 0) return fail(LSX_E_INVALID, "max_wavepackets must be >= 0");
  if (std::isnan(desc->band_tol)) return fail(LSX_E_INVALID, "band_tol must not be NaN");
  lsx_plan* pl = nullptr;
  LSX_TRY(plan_create(sys, desc->tau, desc->scheme, desc->kappa, desc->precision, desc->band_tol, stream, &pl));
  pl->max_w = desc->max_wavepackets;
  *out = pl;
  return LSX_OK;
}

extern "C" lsx_status lsx_plan_propagator(const lsx_plan* pl, int32_t layer, int32_t half, int32_t fibre,
                                          double* out, void* stream) {
  if (!pl || !out) return fail(LSX_E_INVALID, "null argument");
  if (layer < 1 || layer > pl->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (half < 0 || half > 2) return fail(LSX_E_INVALID, "slot must be 0, 1 or 2");
  const LayerDev& ld = pl->L[layer - 1];
  if (fibre < 0 || fibre >= ld.nf) return fail(LSX_E_INVALID, "fibre out of range");
  const PropSet& ps = ld.prop[half];
  if (!ps.present) return fail(LSX_E_INVALID, "plan holds no propagator for this layer/half");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int L = ld.h_ptr[fibre + 1] - ld.h_ptr[fibre];
  const int64_t bytes = prop_bytes(pl->fmt, L);
  std::vector<char> raw(bytes);
  LSX_HIP_TRY(hipMemcpyAsync(raw.data(), ps.data.p + ps.h_off[fibre], bytes, hipMemcpyDeviceToHost, s));
  std::vector<double2> dg;
  if (pl->fmt != PF_F64) {
    dg.resize(L);
    const double2* src = pl->diag.p + (size_t)((layer - 1) * 3 + half) * pl->sys->N + ld.h_d0[fibre];
    LSX_HIP_TRY(hipMemcpyAsync(dg.data(), src, L * sizeof(double2), hipMemcpyDeviceToHost, s));
  }
  LSX_HIP_TRY(hipStreamSynchronize(s));
  // row a of the stored propagator (the plan's order) is row sg[a] of the fibre in the system's
  // order (rows ascending)
  std::vector<int> sg(L);
  {
    const int r0 = ld.h_ptr[fibre];
    const std::vector<int32_t>& sr = pl->sys->fib[layer - 1].rows;
    for (int a = 0; a < L; ++a)
      sg[a] = (int)(std::lower_bound(sr.begin() + r0, sr.begin() + r0 + L, ld.h_rows[r0 + a]) - (sr.begin() + r0));
  }
  auto bf = [](uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
  };
  for (int a = 0; a < L; ++a)
    for (int b = 0; b < L; ++b) {
      double re, im;
      if (pl->fmt == PF_F64 || pl->fmt == PF_F32) {
        const int Lp = round_up(L, 16);
        const int64_t idx = ((int64_t)(a / 16) * (Lp / 4) + b / 4) * 64 + (a % 16) + 16 * (b % 4);
        if (pl->fmt == PF_F64) {
          const double* p = reinterpret_cast<const double*>(raw.data()) + 2 * idx;
          re = p[0];
          im = p[1];
        } else {
          const float* p = reinterpret_cast<const float*>(raw.data()) + 2 * idx;
          re = p[0];
          im = p[1];
        }
      } else {
        const int Lp = round_up(L, 32);
        const int64_t chunk = (int64_t)(a / 16) * (Lp / 32) + b / 32;
        const int lane = (a % 16) + 16 * ((b % 32) / 8), el = b % 8;
        const uint16_t* q = reinterpret_cast<const uint16_t*>(raw.data());
        re = im = 0.0;
        for (int term = 0; term < 3; ++term) {
          re += bf(q[((chunk * 6 + 2 * term) * 64 + lane) * 8 + el]);
          im += bf(q[((chunk * 6 + 2 * term + 1) * 64 + lane) * 8 + el]);
        }
      }
      if (pl->fmt != PF_F64 && a == b) {
        re = dg[a].x;
        im = dg[a].y;
      }
      out[2 * ((int64_t)sg[a] * L + sg[b])] = re;
      out[2 * ((int64_t)sg[a] * L + sg[b]) + 1] = im;
    }
  return LSX_OK;
}

extern "C" lsx_status lsx_plan_sharing(const lsx_plan* pl, int32_t layer, int32_t* ndistinct, int32_t* nsym) {
  if (!pl) return fail(LSX_E_INVALID, "null plan");
  if (layer < 1 || layer > pl->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (ndistinct) *ndistinct = pl->L[layer - 1].nunique;
  if (nsym) *nsym = pl->nsym;
  return LSX_OK;
}

extern "C" lsx_status lsx_plan_band(const lsx_plan* pl, int32_t layer, double* tol, int64_t* kept,
                                    int64_t* dense, int64_t* stored_kept, int64_t* stored_rows) {
  if (!pl) return fail(LSX_E_INVALID, "null plan");
  if (layer < 1 || layer > pl->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  const LayerDev& ld = pl->L[layer - 1];
  int64_t k = 0, d = 0, sk = 0, sr = 0;
  std::vector<char> seen(ld.nunique, 0);
  for (int f = 0; f < ld.nf; ++f) {
    const int L = ld.h_ptr[f + 1] - ld.h_ptr[f];
    const bool first = !seen[ld.rep[f]];
    seen[ld.rep[f]] = 1;
    d += (int64_t)L * L;
    if (first) sr += L;
    for (int rb = 0; rb < (L + 15) / 16; ++rb) {
      int32_t k0, k1;
      fibre_band(ld, f, rb, 1, k0, k1);
      const int64_t e = (int64_t)std::min(16, L - 16 * rb) * (std::min(k1, L) - k0);
      k += e;
      if (first) sk += e;
    }
  }
  if (tol) *tol = pl->band_tol;
  if (kept) *kept = k;
  if (dense) *dense = d;
  if (stored_kept) *stored_kept = sk;
  if (stored_rows) *stored_rows = sr;
  return LSX_OK;
}

extern "C" lsx_status lsx_plan_fibre_band(const lsx_plan* pl, int32_t layer, int32_t fibre, int32_t* lo_hi) {
  if (!pl || !lo_hi) return fail(LSX_E_INVALID, "null argument");
  if (layer < 1 || layer > pl->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  const LayerDev& ld = pl->L[layer - 1];
  if (fibre < 0 || fibre >= ld.nf) return fail(LSX_E_INVALID, "fibre out of range");
  const int L = ld.h_ptr[fibre + 1] - ld.h_ptr[fibre];
  for (int rb = 0; rb < (L + 15) / 16; ++rb) {
    int32_t k0, k1;
    fibre_band(ld, fibre, rb, 1, k0, k1);
    lo_hi[2 * rb] = k0;
    lo_hi[2 * rb + 1] = std::min(k1, round_up(L, prop_pad(pl->fmt)));
  }
  return LSX_OK;
}

extern "C" lsx_status lsx_plan_destroy(lsx_plan* pl) {
  if (!pl) return LSX_OK;
  if (pl->nstates > 0) return fail(LSX_E_STATE, "plan still has live states");
  pl->sys->nplans--;
  delete pl;
  return LSX_OK;
}

// ================================================================ state
struct lsx_state {
  lsx_plan* plan = nullptr;
  int W = 0;
  double2* buf[2] = {nullptr, nullptr};
  bool owns0 = false;
  DBuf<double2> own0, work;
  DBuf<TileDesc> tiles[kMaxLayers];
  int ntiles[kMaxLayers] = {0, 0, 0};
  int nb[kMaxLayers] = {1, 1, 1}, ks[kMaxLayers] = {4, 4, 4};  // tile shape per layer (16*nb columns, ks waves split k)
  int u[kMaxLayers] = {0, 0, 0};       // K-split FP64/FP32: k-step groups in flight per wave (0: default)
  float tuned_us[kMaxLayers] = {0.f, 0.f, 0.f};                // measured pass time of the chosen shape (0: not tuned)
  // runner-up tile shape per layer from the single-pass timings (alt_nb = 0: none); the
  // step-like cycle may prefer it
  int alt_nb[kMaxLayers] = {0, 0, 0}, alt_ks[kMaxLayers] = {0, 0, 0}, alt_u[kMaxLayers] = {0, 0, 0};
  int alt_ntiles[kMaxLayers] = {0, 0, 0};
  float alt_us[kMaxLayers] = {0.f, 0.f, 0.f};
  DBuf<TileDesc> alt_tiles[kMaxLayers];
  int nt = 0;                          // pass output stores: 0 ordinary, 1 non-temporal
  float store_us[2] = {0.f, 0.f};      // measured time of a step-like pass cycle per store mode
  DBuf<double> partial, result;
  int nred = 0;
  int nbatches = 0;                    // batches that reference this state
  int nsamplers = 0;                   // samplers that reference this state
  // lsx_step: captured graphs of the repeated step body (StepGraph::k repetitions each), one per
  // arrangement of the two arrays (an owned state's arrays swap roles after an odd number of
  // passes); dropped whenever the tile shapes or the store mode change
  // captured step graphs, one per (arrangement of the two arrays, body repetitions): the sizes
  // of one call's ladder for each of the arrangements a call can start from
  struct StepGraph {
    double2* b0 = nullptr;
    int cur = 0, lay = 0;
    int64_t k = 0;
    uint64_t used = 0;  // last use (the least recently used one is replaced when all are taken)
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
  };
  static constexpr int kMaxStepGraphs = 16;
  StepGraph sg[kMaxStepGraphs];
  uint64_t graph_clock = 0;
  hipStream_t cap = nullptr;
  static void release(StepGraph& x) {
    if (x.e) (void)hipGraphExecDestroy(x.e);
    if (x.g) (void)hipGraphDestroy(x.g);
    x = StepGraph{};
  }
  // replays still running finish first (the graphs are released on the host's order)
  void drop_graphs() {
    bool any = false;
    for (const StepGraph& x : sg) any = any || x.e;
    if (any) (void)hipDeviceSynchronize();
    for (StepGraph& x : sg) release(x);
  }
  ~lsx_state() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// Passes per captured step graph: a graph launch costs about as much as a dozen kernel
// launches, and kernels inside one graph follow each other faster than host-issued launches,
// so a graph holds many repetitions of the step body (LSX_GRAPH_PASSES overrides the size).
// A single state's call replays graphs of kGraphPasses passes for its bulk and halved sizes
// down to kGraphMinPasses (LSX_GRAPH_MIN_PASSES) for the remainder; a batch replays graphs of
// kBatchGraphPasses.
static constexpr int kGraphPasses = 512;
static constexpr int kGraphMinPasses = 32;
static constexpr int kBatchGraphPasses = 128;
static int64_t graph_passes(int dflt) { return std::max(1, env_int("LSX_GRAPH_PASSES", dflt)); }
static int64_t graph_min_passes() { return std::max(1, env_int("LSX_GRAPH_MIN_PASSES", kGraphMinPasses)); }
// Graph replay pays where the passes are launch-bound: a captured graph starts consecutive
// kernels sooner than host launches do, which matters for passes of a few microseconds, while
// on passes of tens of microseconds and more it measured equal or slower.  By default
// (LSX_GRAPH unset) graphs are used when every layer's tuned pass takes at most kGraphMaxUs;
// LSX_GRAPH=1 always uses them, LSX_GRAPH=0 never.
static constexpr float kGraphMaxUs = 20.f;
static bool use_step_graphs(const float* tuned_us, int nl) {
  const int mode = env_int("LSX_GRAPH", -1);
  if (mode >= 0) return mode != 0;
  for (int l = 0; l < nl; ++l)
    if (!(tuned_us[l] > 0.f && tuned_us[l] <= kGraphMaxUs)) return false;
  return true;
}


// Tile order of one fibre pass.  Workgroup i of a launch runs on XCD i % 8, and each XCD has
// its own L2, so fibres are assigned to XCDs whole (longest first, to the least-loaded XCD) and
// the XCD queues are interleaved; every queue lists its largest tiles first.  Fibres that share
// one stored propagator (point-symmetry orbits, kappa = 1 windows) go to the same XCD in groups
// of up to kOrbitMax, with the tiles of a group's fibres for the same rows and columns listed
// back to back, so each propagator block is fetched into that L2 once for the whole group
// (LSX_GROUP_TILES=0 assigns every fibre on its own).  orbit: single-state orbit tiles, one per
// group and row block (f = the group's entry in the layer's orbit table), which multiply the
// group's states together.  Shorter queues are padded with empty tiles (f = -1).  ms > 1:
// tiles of the row-split kernels, rb counts groups of ms 16-row blocks.
static void build_tiles(const lsx_plan* pl, int layer, int W, int nb, int wb0, int wb1, std::vector<TileDesc>& out,
                        int ms = 1, bool orbit = false) {
  const LayerDev& ld = pl->L[layer - 1];
  const int wt = wb1 - wb0;
  (void)W;
  (void)nb;
  const int NX = std::max(1, env_int("LSX_XCDS", 8));
  const bool share = orbit || (env_int("LSX_GROUP_TILES", 1) != 0 && (int)ld.groups.size() > 0);
  std::vector<std::vector<int>> single;
  if (!share) {
    single.resize(ld.nf);
    for (int f = 0; f < ld.nf; ++f) single[f] = {f};
  }
  const std::vector<std::vector<int>>& groups = share ? ld.groups : single;
  auto glen = [&](const std::vector<int>& g) { return ld.h_ptr[g[0] + 1] - ld.h_ptr[g[0]]; };
  std::vector<int> order(groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return glen(groups[x]) > glen(groups[y]); });
  // balance the bins by tile count (equal counts need no padding tiles), ties by cost
  std::vector<double> load(NX, 0.0);
  std::vector<int64_t> count(NX, 0);
  std::vector<std::vector<TileDesc>> bins(NX);
  for (int gi : order) {
    const std::vector<int>& g = groups[gi];
    const int L = glen(g);
    const int nrb = ((L + 15) / 16 + ms - 1) / ms;
    const int ntg = orbit ? 1 : (int)g.size();  // tiles per row block and column block
    int x = 0;
    for (int y = 1; y < NX; ++y)
      if (count[y] < count[x] || (count[y] == count[x] && load[y] < load[x])) x = y;
    count[x] += (int64_t)nrb * wt * ntg;
    for (int rb = 0; rb < nrb; ++rb) {
      for (int wb = wb0; wb < wb1; ++wb) {
        for (int i = 0; i < ntg; ++i) {
          const int f = g[i];
          int32_t k0, k1;
          fibre_band(ld, f, rb * ms, ms, k0, k1);
          if (wb == wb0) load[x] += (double)wt * (std::min(k1, L) - k0 + 8) * (orbit ? (double)g.size() : 1.0);
          TileDesc t;
          t.r0 = ld.h_ptr[f];
          t.L = L;
          t.rb = rb;
          t.wb = wb;
          t.poff = ld.h_poff.empty() ? 0 : ld.h_poff[f];
          t.f = orbit ? gi : f;
          t.d0 = ld.h_d0.empty() ? ld.h_ptr[f] : ld.h_d0[f];
          t.k0 = k0;
          t.k1 = k1;
          t.bb = ld.h_boff.empty() ? -1 : (int32_t)ld.h_boff[ld.rep[f]];
          t.pad_ = 0;
          bins[x].push_back(t);
        }
      }
    }
  }
  TileDesc empty{};
  empty.f = -1;
  size_t maxlen = 0;
  for (auto& b : bins) maxlen = std::max(maxlen, b.size());
  out.clear();
  for (size_t i = 0; i < maxlen; ++i)
    for (int x = 0; x < NX; ++x) out.push_back(i < bins[x].size() ? bins[x][i] : empty);
  while (!out.empty() && out.back().f < 0) out.pop_back();
}


// Store mode of the pass outputs, prefetch depth and tile shape, in the setting of a step.  A
// step's passes each read the previous pass's output in their own layer's fibre order, written
// mostly by other XCDs; whether ordinary or non-temporal stores make that hand-over faster
// depends on the state's size relative to the caches, and which tile shape and how many k-step
// groups in flight suit a layer depend on where its operands come from (single-pass timings
// read them from the same XCD's L2).  So a cycle of passes over the layers in step order
// (layer j reads its fibre order and writes layer j+1's) is timed with both store modes, for
// the single-pass winner of every layer and, one layer at a time, for its alternatives: the
// winner with the other depth (where a depth was tuned) and the single-pass runner-up.  The
// cycle runs between the work array and a scratch array of the same size, so the state is not
// modified.  Without room for the scratch array everything stays as the single passes chose.
// With tune_store false the store mode stays as set (ordinary or forced).
static lsx_status choose_cycle(lsx_plan* pl, lsx_state* st, bool tune_store) {
  const int nl = pl->sys->nl, W = st->W;
  const int64_t N = pl->sys->N;
  DBuf<double2> tmp;
  if (tmp.alloc((size_t)N * W) != LSX_OK) return LSX_OK;
  PassArgs a[kMaxLayers];
  for (int layer = 1; layer <= nl; ++layer) {
    const LayerDev& ld = pl->L[layer - 1];
    int slot = 0;
    while (slot < 2 && !ld.prop[slot].present) ++slot;
    if (!ld.prop[slot].present) return fail(LSX_E_STATE, "internal: layer without propagators");
    PassArgs& x = a[layer - 1];
    x.out_pos = layout_map(pl, layer, layer % nl + 1);
    x.P = ld.prop[slot].data.p;
    x.diag = pl->diag.p ? pl->diag.p + (size_t)((layer - 1) * 3 + slot) * N : nullptr;
    x.zero = pl->zero.p;
    x.rb_band = ld.d_band.p;
    x.orbit = ld.d_orbit.p;
    x.orbit_max = ld.orbit_max;
    x.W = W;
  }
  // per layer: option 0 the single-pass winner, 1 the winner at the other depth, 2 the runner-up
  struct Opt {
    bool ok;
    int nb, ks, u, ntiles;
    const TileDesc* tiles;
  };
  Opt opt[kMaxLayers][3];
  for (int l = 0; l < nl; ++l) {
    opt[l][0] = {true, st->nb[l], st->ks[l], st->u[l], st->ntiles[l], st->tiles[l].p};
    opt[l][1] = {st->u[l] == 1 || st->u[l] == 2, st->nb[l], st->ks[l], 3 - st->u[l], st->ntiles[l], st->tiles[l].p};
    opt[l][2] = {st->alt_nb[l] > 0, st->alt_nb[l], st->alt_ks[l], st->alt_u[l], st->alt_ntiles[l], st->alt_tiles[l].p};
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(LSX_E_HIP, "event creation failed");
  }
  hipError_t he = hipSuccess;
  int pick[kMaxLayers] = {0, 0, 0};
  auto cycle = [&](int nt) {
    double2* src = st->buf[1];
    double2* dst = tmp.p;
    for (int l = 0; l < nl && he == hipSuccess; ++l) {
      const Opt& o = opt[l][pick[l]];
      PassArgs x = a[l];
      x.tiles = o.tiles;
      x.X = src;
      x.Y = dst;
      x.nt = nt;
      x.u = o.u;
      he = launch_pass(nullptr, pl->fmt, W, o.ntiles, o.nb, o.ks, x);
      std::swap(src, dst);
    }
  };
  auto timed = [&](int nt, int reps) {
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && he == hipSuccess; ++r) cycle(nt);
    if (he == hipSuccess) he = hipEventRecord(e1, nullptr);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    return ms * 1e3f / reps;
  };
  if (tune_store) st->store_us[0] = st->store_us[1] = 0.f;
  // the cycle with the current picks, each store mode: about 5 ms of passes, 3 to 500 cycles
  // sized by a timed warm-up cycle (a few-microsecond cycle needs many for a stable ranking);
  // returns the best time and its mode
  auto evaluate = [&](int& nt_best) {
    float best = -1.f;
    for (int m = 0; m < (tune_store ? 2 : 1) && he == hipSuccess; ++m) {
      const int nt = tune_store ? m : st->nt;
      const float warm_us = timed(nt, 1);
      const int reps = (int)std::max(3.0, std::min(500.0, 5000.0 / std::max(1.0f, warm_us)));
      const float us = timed(nt, reps);
      if (tune_store && (st->store_us[nt] == 0.f || us < st->store_us[nt])) st->store_us[nt] = us;
      if (best < 0.f || us < best) {
        best = us;
        nt_best = nt;
      }
    }
    return best;
  };
  int best_nt = st->nt;
  float best = evaluate(best_nt);
  int best_pick[kMaxLayers] = {0, 0, 0};
  for (int l = 0; l < nl && he == hipSuccess; ++l)
    for (int k = 1; k < 3 && he == hipSuccess; ++k) {
      if (!opt[l][k].ok) continue;
      for (int j = 0; j < nl; ++j) pick[j] = best_pick[j];
      pick[l] = k;
      int nt = best_nt;
      const float us = evaluate(nt);
      if (he == hipSuccess && us < best) {
        best = us;
        best_nt = nt;
        for (int j = 0; j < nl; ++j) best_pick[j] = pick[j];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (he != hipSuccess) return fail(LSX_E_HIP, std::string("step-cycle tuning: ") + hipGetErrorString(he));
  st->nt = best_nt;
  for (int l = 0; l < nl; ++l) {
    if (best_pick[l] == 1) {
      st->u[l] = opt[l][1].u;
    } else if (best_pick[l] == 2) {  // install the runner-up; the former winner becomes it
      std::swap(st->nb[l], st->alt_nb[l]);
      std::swap(st->ks[l], st->alt_ks[l]);
      std::swap(st->u[l], st->alt_u[l]);
      std::swap(st->ntiles[l], st->alt_ntiles[l]);
      std::swap(st->tuned_us[l], st->alt_us[l]);
      std::swap(st->tiles[l].p, st->alt_tiles[l].p);
      std::swap(st->tiles[l].n, st->alt_tiles[l].n);
    }
  }
  return LSX_OK;
}

// Tile shape per layer.  LSX_NB / LSX_KS force a shape; otherwise, unless
// LSX_AUTOTUNE=0, every candidate shape is timed on this state's own size (reading the
// state array, writing only the work array, so the state is not modified) and the
// fastest one per layer is kept.
// Row-split shapes the kernels are built for: m waves on consecutive row blocks sharing the
// staged state of 16 nb columns (mixed formats; FP32 needs m <= 4 nb, BF16x3 nb <= 2).
static bool rowsplit_shape(int fmt, int nb, int m) {
  if (fmt == PF_F64 || !(m == 2 || m == 4 || m == 8)) return false;
  if (fmt == PF_BF16X3) return nb == 1 || nb == 2;
  return (nb == 1 || nb == 2 || nb == 4) && m <= 4 * nb;
}

static lsx_status choose_tiles(lsx_plan* pl, lsx_state* st) {
  const int W = st->W;
  // ks > 0: ks waves split the fibre length; ks < 0: -ks waves take consecutive row blocks
  // and share the LDS-staged state operand (mixed FP32 and BF16x3 paths, BF16x3 with nb <= 2)
  // u: groups of k-steps each wave of a K-split FP64 / FP32 tile keeps in flight (0: the
  // library default, LSX_PREFETCH); shorter fibres favour 1 (fewer registers, more waves)
  struct Shape {
    int nb, ks, u;
  };
  std::vector<Shape> cands;
  const int fnb = env_int("LSX_NB", 0), fks = env_int("LSX_KS", 0);
  const bool tune_u = (pl->fmt == PF_F64 || pl->fmt == PF_F32) && std::getenv("LSX_PREFETCH") == nullptr;
  if (W == 1) {
    // ks < 0: tiles of four row blocks, one row per lane, -ks waves; nb = kOrbitNB: orbit tiles
    // (layers whose fibres share propagators)
    for (int nb : {1, kOrbitNB})
      for (int k : {1, 2, 4, 8}) {
        if (k < 8) cands.push_back({nb, k, 0});
        cands.push_back({nb, -k, 0});
      }
  } else {
    for (int nb : {1, 2, 4})
      for (int k : {1, 2, 4})
        if (16 * nb <= round_up(W, 16) && !(nb == 4 && k == 4)) {
          cands.push_back({nb, k, tune_u ? 2 : 0});
          if (tune_u) cands.push_back({nb, k, 1});
        }
    if (pl->fmt == PF_F32 || pl->fmt == PF_BF16X3)
      for (int nb : {1, 2, 4})
        for (int m : {2, 4, 8})
          if (16 * nb <= round_up(W, 16) && rowsplit_shape(pl->fmt, nb, m)) cands.push_back({nb, -m, 0});
  }
  if (fnb > 0 || fks != 0) {
    const bool rowsplit = fks < 0 && ((W > 1 && rowsplit_shape(pl->fmt, fnb > 0 ? fnb : 1, -fks)) ||
                                      (W == 1 && (fks == -1 || fks == -2 || fks == -4 || fks == -8)));
    const Shape f{(fnb == 1 || fnb == 2 || fnb == 4 || (W == 1 && fnb == kOrbitNB)) ? fnb : 1,
                  rowsplit ? fks : ((fks == 1 || fks == 2 || fks == 4) ? fks : 2), 0};
    cands.assign(1, f);
  } else if (env_int("LSX_AUTOTUNE", 1) == 0 || pl->sys->N == 0) {
    cands.assign(1, Shape{1, W == 1 ? 4 : 2, 0});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timing = cands.size() > 1;
  if (timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(LSX_E_HIP, "event creation failed");
  }
  lsx_status err = LSX_OK;
  const int nl = pl->sys->nl;
  for (int layer = 1; layer <= nl && err == LSX_OK; ++layer) {
    float best = -1.f, second = -1.f;
    st->alt_nb[layer - 1] = 0;
    for (Shape c : cands) {
      if (W == 1 && c.nb == kOrbitNB && pl->L[layer - 1].orbit_max < 2) {
        if (cands.size() > 1) continue;  // no fibre of this layer shares its propagator
        c.nb = 1;
      }
      std::vector<TileDesc> t;
      const int wt = (W == 1) ? 1 : (W + 16 * c.nb - 1) / (16 * c.nb);
      // row blocks per tile: W = 1 four for ks < 0 (one row per lane), else -ks for the row-split shapes
      build_tiles(pl, layer, W, c.nb, 0, wt, t, c.ks < 0 ? (W == 1 ? 4 : -c.ks) : 1, W == 1 && c.nb == kOrbitNB);
      DBuf<TileDesc> d;
      if ((err = d.upload(t, nullptr)) != LSX_OK) break;
      float ms = 0.f;
      if (timing) {
        // steady-state access pattern of the step: fibre-contiguous read, scattered write
        // into the next layer's order, with the first propagator slot the plan holds
        const LayerDev& ld = pl->L[layer - 1];
        int slot = 0;
        while (slot < 2 && !ld.prop[slot].present) ++slot;
        if (!ld.prop[slot].present) {
          err = fail(LSX_E_STATE, "internal: layer without propagators");
          break;
        }
        PassArgs a;
        a.tiles = d.p;
        a.in_pos = nullptr;
        a.out_pos = layout_map(pl, layer, layer % nl + 1);
        a.ph_idx = nullptr;
        a.ph = nullptr;
        a.P = ld.prop[slot].data.p;
        a.diag = pl->diag.p ? pl->diag.p + (size_t)((layer - 1) * 3 + slot) * pl->sys->N : nullptr;
        a.X = st->buf[0];
        a.Y = st->buf[1];
        a.zero = pl->zero.p;
        a.rb_band = ld.d_band.p;
        a.orbit = ld.d_orbit.p;
        a.orbit_max = ld.orbit_max;
        a.W = W;
        a.u = c.u;
        // two timed passes (enough for passes of a millisecond or more), then, for shorter
        // passes, at least five and about 1 ms of them: launch jitter is comparable to a
        // few-microsecond pass
        auto time_reps = [&](int reps, float& per) {
          hipError_t e = hipEventRecord(e0, nullptr);
          for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_pass(nullptr, pl->fmt, W, (int)t.size(), c.nb, c.ks, a);
          if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float total = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&total, e0, e1);
          per = total / reps;
          return e;
        };
        hipError_t he = launch_pass(nullptr, pl->fmt, W, (int)t.size(), c.nb, c.ks, a);
        if (he == hipSuccess) he = time_reps(2, ms);
        if (he == hipSuccess && ms < 1.0f) he = time_reps(std::min(100, std::max(5, (int)(1.0f / std::max(ms, 1e-3f)))), ms);
        if (he != hipSuccess) {
          err = fail(LSX_E_HIP, std::string("autotune: ") + hipGetErrorString(he));
          break;
        }
      }
      const int l = layer - 1;
      if (best < 0.f || ms < best) {
        if (best >= 0.f) {  // the previous best becomes the runner-up
          second = best;
          st->alt_nb[l] = st->nb[l];
          st->alt_ks[l] = st->ks[l];
          st->alt_u[l] = st->u[l];
          st->alt_ntiles[l] = st->ntiles[l];
          st->alt_us[l] = best * 1e3f;
          st->alt_tiles[l].release();
          std::swap(st->alt_tiles[l].p, st->tiles[l].p);
          std::swap(st->alt_tiles[l].n, st->tiles[l].n);
        }
        best = ms;
        st->nb[l] = c.nb;
        st->ks[l] = c.ks;
        st->u[l] = c.u;
        st->tiles[l].release();
        std::swap(st->tiles[l].p, d.p);
        std::swap(st->tiles[l].n, d.n);
        st->ntiles[l] = (int)t.size();
      } else if (second < 0.f || ms < second) {
        second = ms;
        st->alt_nb[l] = c.nb;
        st->alt_ks[l] = c.ks;
        st->alt_u[l] = c.u;
        st->alt_ntiles[l] = (int)t.size();
        st->alt_us[l] = ms * 1e3f;
        st->alt_tiles[l].release();
        std::swap(st->alt_tiles[l].p, d.p);
        std::swap(st->alt_tiles[l].n, d.n);
      }
    }
    st->tuned_us[layer - 1] = timing ? best * 1e3f : 0.f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != LSX_OK) return err;
  const int fnt = env_int("LSX_NT", -1);
  if (fnt == 0 || fnt == 1) st->nt = fnt;
  if (W == 1 || pl->sys->N == 0 || env_int("LSX_AUTOTUNE", 1) == 0) return LSX_OK;
  return choose_cycle(pl, st, !(fnt == 0 || fnt == 1));
}

extern "C" lsx_status lsx_state_create(lsx_plan* pl, int32_t W, void* dev_ptr, lsx_state** out) {
  if (!pl || !out) return fail(LSX_E_INVALID, "null argument");
  if (W < 1 || W > 65536) return fail(LSX_E_INVALID, "W must be in [1, 65536]");
  if (pl->max_w > 0 && W > pl->max_w) return fail(LSX_E_INVALID, "W exceeds the plan's max_wavepackets");
  if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) % 16) != 0)
    return fail(LSX_E_INVALID, "wrapped device pointer must be 16-byte aligned");
  const int64_t N = pl->sys->N;
  lsx_state* st = new (std::nothrow) lsx_state();
  if (!st) return fail(LSX_E_OOM, "host allocation failed");
  st->plan = pl;
  st->W = W;
  auto cleanup = [&](lsx_status e) {
    delete st;
    return e;
  };
  lsx_status e;
  const size_t total = (size_t)std::max<int64_t>(N, 1) * W;
  if (dev_ptr) {
    st->buf[0] = reinterpret_cast<double2*>(dev_ptr);
  } else {
    if ((e = st->own0.alloc(total)) != LSX_OK) return cleanup(e);
    st->buf[0] = st->own0.p;
    st->owns0 = true;
    if (hipMemset(st->buf[0], 0, total * sizeof(double2)) != hipSuccess)
      return cleanup(fail(LSX_E_HIP, "hipMemset of state failed"));
  }
  if ((e = st->work.alloc(total)) != LSX_OK) return cleanup(e);
  st->buf[1] = st->work.p;
  if ((e = choose_tiles(pl, st)) != LSX_OK) return cleanup(e);
  st->nred = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (N + 255) / 256));
  // observables: mass, energy and the fibre masses of every layer in one result block
  size_t nfsum = 0;
  for (int j = 0; j < pl->sys->nl; ++j) nfsum += (size_t)pl->L[j].nf;
  if ((e = st->partial.alloc((size_t)st->nred * W)) != LSX_OK) return cleanup(e);
  if ((e = st->result.alloc((size_t)W * (2 + std::max<size_t>(nfsum, 1)))) != LSX_OK) return cleanup(e);
  if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(LSX_E_HIP, "state setup failed"));
  pl->nstates++;
  *out = st;
  return LSX_OK;
}

extern "C" lsx_status lsx_state_wrap(lsx_plan* pl, int32_t W, void* dev_ptr, lsx_state** out) {
  if (!dev_ptr) return fail(LSX_E_INVALID, "null device pointer");
  return lsx_state_create(pl, W, dev_ptr, out);
}

extern "C" lsx_status lsx_state_upload(lsx_state* st, const double* host, void* stream) {
  if (!st || !host) return fail(LSX_E_INVALID, "null argument");
  const size_t bytes = (size_t)st->plan->sys->N * st->W * sizeof(double2);
  if (bytes)
    LSX_HIP_TRY(hipMemcpyAsync(st->buf[0], host, bytes, hipMemcpyHostToDevice, reinterpret_cast<hipStream_t>(stream)));
  return LSX_OK;
}

extern "C" lsx_status lsx_state_download(lsx_state* st, double* host, void* stream) {
  if (!st || !host) return fail(LSX_E_INVALID, "null argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)st->plan->sys->N * st->W * sizeof(double2);
  if (bytes) LSX_HIP_TRY(hipMemcpyAsync(host, st->buf[0], bytes, hipMemcpyDeviceToHost, s));
  LSX_HIP_TRY(hipStreamSynchronize(s));
  return LSX_OK;
}

extern "C" lsx_status lsx_state_device_ptr(const lsx_state* st, void** dev) {
  if (!st || !dev) return fail(LSX_E_INVALID, "null argument");
  *dev = st->buf[0];
  return LSX_OK;
}

extern "C" lsx_status lsx_state_tuning(const lsx_state* st, int32_t layer, int32_t* nb, int32_t* ks,
                                       double* pass_us) {
  if (!st) return fail(LSX_E_INVALID, "null state");
  if (layer < 1 || layer > st->plan->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (nb) *nb = st->nb[layer - 1];
  if (ks) *ks = st->ks[layer - 1];
  if (pass_us) *pass_us = st->tuned_us[layer - 1];
  return LSX_OK;
}

extern "C" lsx_status lsx_state_prefetch(const lsx_state* st, int32_t layer, int32_t* groups) {
  if (!st) return fail(LSX_E_INVALID, "null state");
  if (layer < 1 || layer > st->plan->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (groups) *groups = st->u[layer - 1];
  return LSX_OK;
}

extern "C" lsx_status lsx_state_store_mode(const lsx_state* st, int32_t* nontemporal, double* cycle_us) {
  if (!st) return fail(LSX_E_INVALID, "null state");
  if (nontemporal) *nontemporal = st->nt;
  if (cycle_us) {
    cycle_us[0] = st->store_us[0];
    cycle_us[1] = st->store_us[1];
  }
  return LSX_OK;
}

// Tile shapes the pass kernels are built for (see choose_tiles and launch_pass).
static bool shape_valid(int fmt, int W, int nb, int ks, int u) {
  if (W == 1) {
    if ((nb != 1 && nb != kOrbitNB) || u != 0) return false;
    if (ks == 1 || ks == 2 || ks == 4) return true;
    return ks == -1 || ks == -2 || ks == -4 || ks == -8;
  }
  if (!(nb == 1 || nb == 2 || nb == 4) || 16 * nb > round_up(W, 16)) return false;
  if (ks == 1 || ks == 2 || ks == 4)
    return u == 0 || ((fmt == PF_F64 || fmt == PF_F32) && (u == 1 || u == 2));
  if (ks < 0) return u == 0 && rowsplit_shape(fmt, nb, -ks);
  return false;
}

extern "C" lsx_status lsx_state_set_tuning(lsx_state* st, int32_t layer, int32_t nb, int32_t ks, int32_t groups) {
  if (!st) return fail(LSX_E_INVALID, "null state");
  lsx_plan* pl = st->plan;
  if (layer < 1 || layer > pl->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (!shape_valid(pl->fmt, st->W, nb, ks, groups))
    return fail(LSX_E_INVALID, "tile shape not available for this precision and W");
  const int W = st->W;
  const bool orbit = W == 1 && nb == kOrbitNB;
  if (orbit && pl->L[layer - 1].orbit_max < 2)
    return fail(LSX_E_INVALID, "orbit tiles need fibres that share a stored propagator");
  const int wt = (W == 1) ? 1 : (W + 16 * nb - 1) / (16 * nb);
  std::vector<TileDesc> t;
  build_tiles(pl, layer, W, nb, 0, wt, t, ks < 0 ? (W == 1 ? 4 : -ks) : 1, orbit);
  DBuf<TileDesc> d;
  LSX_TRY(d.upload(t, nullptr));
  const int l = layer - 1;
  st->tiles[l].release();
  std::swap(st->tiles[l].p, d.p);
  std::swap(st->tiles[l].n, d.n);
  st->ntiles[l] = (int)t.size();
  st->nb[l] = nb;
  st->ks[l] = ks;
  st->u[l] = groups;
  st->tuned_us[l] = 0.f;
  st->drop_graphs();
  return LSX_OK;
}

extern "C" lsx_status lsx_state_set_store_mode(lsx_state* st, int32_t nontemporal) {
  if (!st) return fail(LSX_E_INVALID, "null state");
  if (nontemporal != 0 && nontemporal != 1) return fail(LSX_E_INVALID, "store mode must be 0 or 1");
  st->nt = nontemporal;
  st->drop_graphs();
  return LSX_OK;
}

extern "C" lsx_status lsx_state_destroy(lsx_state* st) {
  if (!st) return LSX_OK;
  if (st->nbatches > 0) return fail(LSX_E_STATE, "state is still part of a batch");
  if (st->nsamplers > 0) return fail(LSX_E_STATE, "state still has a sampler");
  st->plan->nstates--;
  delete st;
  return LSX_OK;
}

// ================================================================ step composer
// Between API calls the state lives in buf[0] in canonical order.  A fibre pass reads
// buf[cur] and writes buf[1-cur].  Array layouts: layout j = layer-j fibre order, layout nl =
// canonical (the last layer's fibres are contiguous runs).  A pass writes the layout the next
// pass reads fibre-contiguously, so only the first pass of a call gathers through an index
// table; the last pass writes canonical order.  The kinetic phase that follows a pass is
// applied in that pass's epilogue.
namespace {
struct Runner {
  lsx_plan* pl;
  lsx_state* st;
  hipStream_t s;
  int cur = 0;
  int lay = 0;  // layout of buf[cur]; 0 = canonical

  const int32_t* table(int layer, int layout) const { return layout_map(pl, layer, layout); }

  // F_layer(t) with t = tau (half 0) or tau/2; `next` is the layer of the following
  // pass (0: none, write canonical order); phase_half >= 0 fuses Phase(kappa t') after it.
  lsx_status pass(int layer, int half, int next, int phase_half) {
    const LayerDev& ld = pl->L[layer - 1];
    const PropSet& ps = ld.prop[half];
    if (!ps.present) return fail(LSX_E_INVALID, "plan holds no propagator for this layer/slot");
    if (phase_half >= 0 && pl->kappa != 0.0 && !pl->phase[phase_half].p)
      return fail(LSX_E_INVALID, "plan holds no phase table for this slot");
    const int outlay = next;  // 0: canonical order
    PassArgs a;
    a.tiles = st->tiles[layer - 1].p;
    a.in_pos = table(layer, lay);
    a.out_pos = table(layer, outlay);
    a.ph_idx = table(layer, 0);
    a.ph = (phase_half >= 0 && pl->kappa != 0.0) ? pl->phase[phase_half].p : nullptr;
    a.P = ps.data.p;
    a.diag = pl->diag.p ? pl->diag.p + (size_t)((layer - 1) * 3 + half) * pl->sys->N : nullptr;
    a.X = st->buf[cur];
    a.Y = st->buf[1 - cur];
    a.zero = pl->zero.p;
    a.rb_band = ld.d_band.p;
    a.orbit = ld.d_orbit.p;
    a.orbit_max = ld.orbit_max;
    a.W = st->W;
    a.nt = st->nt;
    a.u = st->u[layer - 1];
    LSX_HIP_TRY(launch_pass(s, pl->fmt, st->W, st->ntiles[layer - 1], st->nb[layer - 1], st->ks[layer - 1], a));
    cur ^= 1;
    lay = outlay;
    return LSX_OK;
  }
  lsx_status phase(int half) {
    if (pl->kappa == 0.0 || pl->sys->N == 0) return LSX_OK;
    if (!pl->phase[half].p) return fail(LSX_E_INVALID, "plan holds no phase table for this slot");
    LSX_HIP_TRY(launch_phase_apply(s, pl->sys->N, st->W, pl->phase[half].p, st->buf[cur]));
    return LSX_OK;
  }
  lsx_status finish() {
    if (cur != 0) {
      if (st->owns0) {
        // both arrays belong to the library: swap roles instead of copying
        std::swap(st->buf[0], st->buf[1]);
      } else {
        LSX_HIP_TRY(hipMemcpyAsync(st->buf[0], st->buf[1], (size_t)pl->sys->N * st->W * sizeof(double2),
                                   hipMemcpyDeviceToDevice, s));
      }
      cur = 0;
    }
    return LSX_OK;
  }
};
}  // namespace

static lsx_status check_pair(lsx_plan* pl, lsx_state* st) {
  if (!pl || !st) return fail(LSX_E_INVALID, "null argument");
  if (st->plan != pl) return fail(LSX_E_STATE, "state belongs to another plan");
  return LSX_OK;
}

// Runs `body(Runner&)` on the caller's stream and leaves the canonical result in buf[0].
template <typename Body>
static lsx_status run_passes(lsx_plan* pl, lsx_state* st, hipStream_t s, Body body) {
  Runner r{pl, st, s};
  LSX_TRY(body(r));
  return r.finish();
}

namespace {
// One fibre pass of a step sequence: layer, propagator slot, layer of the following pass
// (0: none, write canonical order) and the phase slot fused after it (-1: none).
struct PassSpec {
  int layer, half, next, phase_half;
};

// The passes of nsteps steps of a scheme as head, body (repeated reps times) and tail, with
// the sub-steps of consecutive steps merged where the flows compose (App. A).  Two layers:
//  Strang  : F1(t/2) [Ph F2(t) Ph F1(t)]^(n-1) Ph F2(t) Ph F1(t/2)           (Ph = phase(t/2))
//  Lie     : [F1(t) Ph F2(t)]^n                                               (Ph = phase(t))
//  CN      : [F1(t/2) Ph F2(t) Ph F1(t/2)]^n, unmerged (C(t/2)^2 != C(t), eq. 4.6)
//  Yoshida : S2(g1 t) S2(g0 t) S2(g1 t) per step; inside a step the adjacent F1 halves merge into
//            F1((g1+g0) t/2), between steps into F1(g1 t).  Slots as in scheme_times().
// Every two-layer body has an even number of passes and returns to the layout it started from.
// Three layers (Ph as above):
//  Strang  : F1(t/2) F2(t/2) [Ph F3(t) Ph F2(t/2) F1(t) F2(t/2)]^(n-1) Ph F3(t) Ph F2(t/2) F1(t/2)
//  Lie, BE  : [F1(t) F2(t) Ph F3(t)]^n
//  CN      : [F1(t/2) F2(t/2) Ph F3(t) Ph F2(t/2) F1(t/2)]^n, unmerged
//  Yoshida : the three-layer Strang steps of g1 t, g0 t, g1 t with the F1 halves merged as for
//            two layers (13 passes per step)
void step_sequence(int scheme, int nl, int64_t nsteps, std::vector<PassSpec>& head, std::vector<PassSpec>& body,
                   std::vector<PassSpec>& tail, int64_t& reps) {
  head.clear();
  body.clear();
  tail.clear();
  reps = 0;
  if (nl == 3) {
    if (scheme == LSX_YOSHIDA4) {
      const std::vector<PassSpec> inner = {{2, 0, 3, 0}, {3, 0, 2, 0}, {2, 0, 1, -1}, {1, 2, 2, -1},
                                           {2, 1, 3, 1}, {3, 2, 2, 1}, {2, 1, 1, -1}, {1, 2, 2, -1},
                                           {2, 0, 3, 0}, {3, 0, 2, 0}, {2, 0, 1, -1}};
      head = {{1, 1, 2, -1}};
      body = inner;
      body.push_back({1, 0, 2, -1});
      tail = inner;
      tail.push_back({1, 1, 0, -1});
    } else if (scheme == LSX_STRANG_CN) {
      for (int64_t k = 0; k < nsteps; ++k) {
        const bool last = (k + 1 == nsteps);
        tail.push_back({1, 1, 2, -1});
        tail.push_back({2, 1, 3, 1});
        tail.push_back({3, 0, 2, 1});
        tail.push_back({2, 1, 1, -1});
        tail.push_back({1, 1, last ? 0 : 1, -1});
      }
      return;
    } else if (scheme == LSX_STRANG) {
      head = {{1, 1, 2, -1}, {2, 1, 3, 1}};
      body = {{3, 0, 2, 1}, {2, 1, 1, -1}, {1, 0, 2, -1}, {2, 1, 3, 1}};
      tail = {{3, 0, 2, 1}, {2, 1, 1, -1}, {1, 1, 0, -1}};
    } else {
      // the first step reads canonical order, later ones layer-1 order: as head, so that the
      // repeated body starts and ends in the same layout
      tail = {{1, 0, 2, -1}, {2, 0, 3, 0}, {3, 0, 0, -1}};
      if (nsteps == 1) return;
      head = {{1, 0, 2, -1}, {2, 0, 3, 0}, {3, 0, 1, -1}};
      body = head;
      reps = nsteps - 2;
      return;
    }
    reps = nsteps - 1;
    return;
  }
  if (scheme == LSX_STRANG) {
    head = {{1, 1, 2, 1}};
    body = {{2, 0, 1, 1}, {1, 0, 2, 1}};
    tail = {{2, 0, 1, 1}, {1, 1, 0, -1}};
    reps = nsteps - 1;
  } else if (scheme == LSX_YOSHIDA4) {
    const std::vector<PassSpec> inner = {{2, 0, 1, 0}, {1, 2, 2, 1}, {2, 2, 1, 1}, {1, 2, 2, 0}, {2, 0, 1, 0}};
    head = {{1, 1, 2, 0}};
    body = inner;
    body.push_back({1, 0, 2, 0});
    tail = inner;
    tail.push_back({1, 1, 0, -1});
    reps = nsteps - 1;
  } else if (scheme == LSX_STRANG_CN) {
    for (int64_t k = 0; k < nsteps; ++k) {
      const bool last = (k + 1 == nsteps);
      tail.push_back({1, 1, 2, 1});
      tail.push_back({2, 0, 1, 1});
      tail.push_back({1, 1, last ? 0 : 1, -1});
    }
  } else if (nsteps == 1) {  // Lie with exact or backward-Euler flows
    tail = {{1, 0, 2, 0}, {2, 0, 0, -1}};
  } else {
    head = {{1, 0, 2, 0}, {2, 0, 1, -1}};
    body = {{1, 0, 2, 0}, {2, 0, 1, -1}};
    tail = {{1, 0, 2, 0}, {2, 0, 0, -1}};
    reps = nsteps - 2;
  }
}
}  // namespace

extern "C" lsx_status lsx_step(lsx_plan* pl, lsx_state* st, int64_t nsteps, void* stream) {
  LSX_TRY(check_pair(pl, st));
  if (nsteps < 0) return fail(LSX_E_INVALID, "nsteps must be >= 0");
  if (nsteps == 0 || pl->sys->N == 0) return LSX_OK;
  std::vector<PassSpec> head, body, tail;
  int64_t reps = 0;
  step_sequence(pl->scheme, pl->sys->nl, nsteps, head, body, tail, reps);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // body repetitions per captured graph (the ladder): about graph_passes() passes for the bulk
  // of the call, then halved sizes down to about graph_min_passes() passes for its remainder,
  // each an even number of passes so that a replay ends in the arrays and layout it starts from
  const int64_t nb = std::max<int64_t>(1, (int64_t)body.size());
  auto even = [nb](int64_t k) { return (k * nb) % 2 ? k + 1 : k; };
  std::vector<int64_t> ladder{even(std::max<int64_t>(1, graph_passes(kGraphPasses) / nb))};
  for (int64_t k = ladder[0] / 2; k >= 1; k /= 2) {
    const int64_t ke = even(k);
    if (ke >= ladder.back() || ke * nb < graph_min_passes()) break;
    ladder.push_back(ke);
  }
  // no captured graph inside a caller's own capture of this stream (its launches are captured
  // as they are)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  LSX_HIP_TRY(hipStreamIsCapturing(s, &cs));
  const bool graphs = use_step_graphs(st->tuned_us, pl->sys->nl) && cs == hipStreamCaptureStatusNone && !body.empty() &&
                      reps >= ladder.back();
  return run_passes(pl, st, s, [&](Runner& r) -> lsx_status {
    for (const PassSpec& p : head) LSX_TRY(r.pass(p.layer, p.half, p.next, p.phase_half));
    int64_t left = reps;
    for (const int64_t k : ladder) {
      if (!graphs || left < k) continue;
      lsx_state::StepGraph* g = nullptr;
      for (lsx_state::StepGraph& x : st->sg)
        if (x.e && x.b0 == st->buf[0] && x.cur == r.cur && x.lay == r.lay && x.k == k) g = &x;
      if (!g) {
        // an empty slot, else the least recently used graph (its replays finish first)
        g = &st->sg[0];
        for (lsx_state::StepGraph& x : st->sg)
          if (!x.e || (g->e && x.used < g->used)) g = &x;
        if (g->e) {
          LSX_HIP_TRY(hipDeviceSynchronize());
          lsx_state::release(*g);
        }
        if (!st->cap) LSX_HIP_TRY(hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking));
        Runner rc{pl, st, st->cap};
        rc.cur = r.cur;
        rc.lay = r.lay;
        LSX_HIP_TRY(hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal));
        lsx_status cap_err = LSX_OK;
        for (int64_t i = 0; i < k && cap_err == LSX_OK; ++i)
          for (const PassSpec& p : body)
            if ((cap_err = rc.pass(p.layer, p.half, p.next, p.phase_half)) != LSX_OK) break;
        hipGraph_t gg = nullptr;
        const hipError_t ee = hipStreamEndCapture(st->cap, &gg);
        if (cap_err == LSX_OK && ee == hipSuccess && (rc.cur != r.cur || rc.lay != r.lay))
          cap_err = fail(LSX_E_STATE, "internal: captured step body does not return to its arrays");
        if (cap_err != LSX_OK || ee != hipSuccess) {
          if (gg) (void)hipGraphDestroy(gg);
          if (cap_err != LSX_OK) return cap_err;
          LSX_HIP_TRY(ee);
        }
        g->g = gg;
        const hipError_t ie = hipGraphInstantiate(&g->e, g->g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
          (void)hipGraphDestroy(g->g);
          *g = lsx_state::StepGraph{};
          LSX_HIP_TRY(ie);
        }
        g->b0 = st->buf[0];
        g->cur = r.cur;
        g->lay = r.lay;
        g->k = k;
      }
      g->used = ++st->graph_clock;
      for (; left >= k; left -= k) LSX_HIP_TRY(hipGraphLaunch(g->e, s));
    }
    for (; left > 0; --left)
      for (const PassSpec& p : body) LSX_TRY(r.pass(p.layer, p.half, p.next, p.phase_half));
    for (const PassSpec& p : tail) LSX_TRY(r.pass(p.layer, p.half, p.next, p.phase_half));
    return LSX_OK;
  });
}

extern "C" lsx_status lsx_fibre_pass(lsx_plan* pl, lsx_state* st, int32_t layer, int32_t half, int32_t count,
                                     void* stream) {
  LSX_TRY(check_pair(pl, st));
  if (layer < 1 || layer > pl->sys->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (half < 0 || half > 2) return fail(LSX_E_INVALID, "slot must be 0, 1 or 2");
  if (count < 0) return fail(LSX_E_INVALID, "count must be >= 0");
  if (pl->sys->N == 0 || count == 0) return LSX_OK;
  return run_passes(pl, st, reinterpret_cast<hipStream_t>(stream), [&](Runner& r) -> lsx_status {
    for (int32_t k = 0; k < count; ++k) LSX_TRY(r.pass(layer, half, k + 1 < count ? layer : 0, -1));
    return LSX_OK;
  });
}

extern "C" lsx_status lsx_phase(lsx_plan* pl, lsx_state* st, int32_t half, void* stream) {
  LSX_TRY(check_pair(pl, st));
  if (half < 0 || half > 2) return fail(LSX_E_INVALID, "slot must be 0, 1 or 2");
  Runner r{pl, st, reinterpret_cast<hipStream_t>(stream)};
  return r.phase(half);
}

extern "C" lsx_status lsx_observables(lsx_plan* pl, lsx_state* st, uint32_t mask, double* out, void* stream) {
  LSX_TRY(check_pair(pl, st));
  if (!out) return fail(LSX_E_INVALID, "null output");
  if (mask == 0 || (mask & ~31u)) return fail(LSX_E_INVALID, "bad observable mask");
  if ((mask & LSX_OBS_FIBRE_MASS_3) && pl->sys->nl < 3) return fail(LSX_E_INVALID, "system has no layer 3");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const lsx_system* sys = pl->sys;
  const int W = st->W;
  const int64_t N = sys->N;
  double* dres = st->result.p;
  size_t count = 0;
  if (mask & LSX_OBS_MASS) {
    LSX_HIP_TRY(launch_reduce(s, 0, N, W, st->buf[0], pl->K2.p, 0, nullptr, nullptr, 0, nullptr, nullptr, 0,
                              nullptr, nullptr, st->partial.p, st->nred, dres + count));
    count += W;
  }
  if (mask & LSX_OBS_ENERGY) {
    const int nv3 = sys->nl > 2 ? sys->pot[2].nv : 0;
    LSX_HIP_TRY(launch_reduce(s, 1, N, W, st->buf[0], pl->K2.p, sys->pot[0].nv, pl->L[0].nbr.p, pl->L[0].v.p,
                              sys->pot[1].nv, pl->L[1].nbr.p, pl->L[1].v.p, nv3, pl->L[2].nbr.p, pl->L[2].v.p,
                              st->partial.p, st->nred, dres + count));
    count += W;
  }
  const uint32_t fm_bit[kMaxLayers] = {LSX_OBS_FIBRE_MASS_1, LSX_OBS_FIBRE_MASS_2, LSX_OBS_FIBRE_MASS_3};
  for (int layer = 1; layer <= sys->nl; ++layer)
    if (mask & fm_bit[layer - 1]) {
      const LayerDev& ld = pl->L[layer - 1];
      LSX_HIP_TRY(launch_fibre_mass(s, ld.nf, ld.ptr.p, ld.rows.p, W, st->buf[0], dres + count));
      count += (size_t)ld.nf * W;
    }
  LSX_HIP_TRY(hipMemcpyAsync(out, dres, count * sizeof(double), hipMemcpyDeviceToHost, s));
  LSX_HIP_TRY(hipStreamSynchronize(s));
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(out[i])) return fail(LSX_E_NONFINITE, "observable is NaN or Inf");
  return LSX_OK;
}

// Allocation-free variant of lsx_observables: the state is a caller-owned device array, the
// results stay on the device, and the reduction partials go to the static scratch array of
// lsx_kernels.hip (one per GPU, shared by every call on that GPU).  The partials are written
// before they are read within a call, so nothing needs clearing; calls that overlap on one GPU
// race on the array.  Same kernels, block count and fixed reduction order as lsx_observables,
// so the two give identical values.
extern "C" lsx_status lsx_observables_noalloc(lsx_plan* pl, const void* dev_c, int32_t W, uint32_t mask,
                                              double* dev_out, void* stream) {
  if (!pl || !dev_c || !dev_out) return fail(LSX_E_INVALID, "null argument");
  if (W < 1 || W > 65536) return fail(LSX_E_INVALID, "W must be in [1, 65536]");
  if (pl->max_w > 0 && W > pl->max_w) return fail(LSX_E_INVALID, "W exceeds the plan's max_wavepackets");
  if (mask == 0 || (mask & ~31u)) return fail(LSX_E_INVALID, "bad observable mask");
  if ((mask & LSX_OBS_FIBRE_MASS_3) && pl->sys->nl < 3) return fail(LSX_E_INVALID, "system has no layer 3");
  const lsx_system* sys = pl->sys;
  const int64_t N = sys->N;
  const int nred = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (N + 255) / 256));
  const bool reduce = (mask & (LSX_OBS_MASS | LSX_OBS_ENERGY)) != 0;
  if (reduce && (int64_t)nred * W > kStaticScratchDoubles)
    return fail(LSX_E_INVALID, "W * min(1024, ceil(N / 256)) = " + std::to_string((int64_t)nred * W) +
                                   " reduction partials exceed the static scratch of " +
                                   std::to_string(kStaticScratchDoubles) + " doubles");
  double* part = nullptr;
  if (reduce) LSX_HIP_TRY(static_scratch(&part));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const double2* c = static_cast<const double2*>(dev_c);
  size_t count = 0;
  if (mask & LSX_OBS_MASS) {
    LSX_HIP_TRY(launch_reduce(s, 0, N, W, c, pl->K2.p, 0, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr,
                              nullptr, part, nred, dev_out + count));
    count += W;
  }
  if (mask & LSX_OBS_ENERGY) {
    const int nv3 = sys->nl > 2 ? sys->pot[2].nv : 0;
    LSX_HIP_TRY(launch_reduce(s, 1, N, W, c, pl->K2.p, sys->pot[0].nv, pl->L[0].nbr.p, pl->L[0].v.p,
                              sys->pot[1].nv, pl->L[1].nbr.p, pl->L[1].v.p, nv3, pl->L[2].nbr.p, pl->L[2].v.p, part,
                              nred, dev_out + count));
    count += W;
  }
  const uint32_t fm_bit[kMaxLayers] = {LSX_OBS_FIBRE_MASS_1, LSX_OBS_FIBRE_MASS_2, LSX_OBS_FIBRE_MASS_3};
  for (int layer = 1; layer <= sys->nl; ++layer)
    if (mask & fm_bit[layer - 1]) {
      const LayerDev& ld = pl->L[layer - 1];
      LSX_HIP_TRY(launch_fibre_mass(s, ld.nf, ld.ptr.p, ld.rows.p, W, c, dev_out + count));
      count += (size_t)ld.nf * W;
    }
  return LSX_OK;
}

// ================================================================ batched systems
namespace {
struct PatternKey {
  int layer, half, inlay, outlay, phase_half, cur;
  bool operator<(const PatternKey& o) const {
    return std::tie(layer, half, inlay, outlay, phase_half, cur) <
           std::tie(o.layer, o.half, o.inlay, o.outlay, o.phase_half, o.cur);
  }
};
}  // namespace

struct lsx_batch {
  std::vector<lsx_plan*> pl;
  std::vector<lsx_state*> st;
  int fmt = 0, scheme = 0;
  bool w1 = false;
  int nl = 2;  // layers of every system in the batch
  DBuf<TileDesc> tiles[kMaxLayers];
  int ntiles[kMaxLayers] = {0, 0, 0};
  int nb[kMaxLayers] = {1, 1, 1}, ks[kMaxLayers] = {2, 2, 2};
  float tuned_us[kMaxLayers] = {0.f, 0.f, 0.f};
  // per pass pattern: the systems' argument array, and whether any system gathers its input
  // through an index table (then the launch uses the gathering kernel for every system)
  std::map<PatternKey, std::pair<std::unique_ptr<DBuf<PassArgs>>, bool>> args;
  std::vector<std::pair<double2*, double2*>> bufs;  // buffers the argument arrays refer to
  DBuf<int32_t> marker;                              // non-null in_pos marker for gathering passes
  DBuf<int32_t> queue;                               // persistent launches: 9 counters, zero between launches
  int u[kMaxLayers] = {0, 0, 0};                     // K-split FP64/FP32: k-step groups in flight (0: 2)
  int persist[kMaxLayers] = {0, 0, 0};               // launch mode per layer: 0 one workgroup per tile,
                                                     // 1 persistent with tile queues, 2 persistent static stride
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int64_t graph_k = 0;  // body repetitions the graph holds
  ~lsx_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// index table of `layer`'s fibre positions inside an array of layout `layout` (two layers)
static const int32_t* layout_table(const lsx_plan* pl, int layer, int layout) {
  return layout_map(pl, layer, layout);
}

// replays still running finish first
static void batch_drop_graph(lsx_batch* b) {
  if (b->exec) (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// per-system argument array of one pass pattern (built once, kept on the device)
static lsx_status batch_args(lsx_batch* b, const PatternKey& k, const PassArgs** out, bool* gather = nullptr) {
  auto it = b->args.find(k);
  if (it == b->args.end()) {
    std::vector<PassArgs> v(b->pl.size());
    bool any = false;
    for (size_t i = 0; i < b->pl.size(); ++i) any = any || layout_table(b->pl[i], k.layer, k.inlay) != nullptr;
    for (size_t i = 0; i < b->pl.size(); ++i) {
      lsx_plan* pl = b->pl[i];
      const lsx_state* st = b->st[i];
      const LayerDev& ld = pl->L[k.layer - 1];
      const PropSet& ps = ld.prop[k.half];
      if (!ps.present) return fail(LSX_E_INVALID, "plan holds no propagator for this layer/half");
      PassArgs& a = v[i];
      a.tiles = nullptr;
      a.in_pos = layout_table(pl, k.layer, k.inlay);
      if (any && !a.in_pos) {
        // the gathering kernel runs for the whole batch: this system gathers through the identity
        if (!pl->iota.p) {
          std::vector<int32_t> id((size_t)std::max<int64_t>(pl->sys->N, 1));
          std::iota(id.begin(), id.end(), 0);
          LSX_TRY(pl->iota.upload(id, nullptr));
        }
        a.in_pos = pl->iota.p;
      }
      a.out_pos = layout_table(pl, k.layer, k.outlay);
      a.ph_idx = layout_map(pl, k.layer, 0);
      a.ph = (k.phase_half >= 0 && pl->kappa != 0.0) ? pl->phase[k.phase_half].p : nullptr;
      a.P = ps.data.p;
      a.diag = pl->diag.p ? pl->diag.p + (size_t)((k.layer - 1) * 3 + k.half) * pl->sys->N : nullptr;
      a.X = st->buf[k.cur];
      a.Y = st->buf[1 - k.cur];
      a.zero = pl->zero.p;
      a.batch = nullptr;
      a.W = st->W;
      a.nt = st->nt;
    }
    auto d = std::make_unique<DBuf<PassArgs>>();
    LSX_TRY(d->alloc(v.size()));
    LSX_HIP_TRY(hipMemcpy(d->p, v.data(), v.size() * sizeof(PassArgs), hipMemcpyHostToDevice));
    it = b->args.emplace(k, std::make_pair(std::move(d), any)).first;
  }
  *out = it->second.first->p;
  if (gather) *gather = it->second.second;
  return LSX_OK;
}

// Tiles of all systems for one layer, f = system index, XCD-interleaved as build_tiles.
static void batch_tiles(const lsx_batch* b, int layer, int nb, std::vector<TileDesc>& out) {
  const int NX = std::max(1, env_int("LSX_XCDS", 8));
  struct Item {
    int sys, f, L;
  };
  std::vector<Item> items;
  for (size_t i = 0; i < b->pl.size(); ++i) {
    const LayerDev& ld = b->pl[i]->L[layer - 1];
    for (int f = 0; f < ld.nf; ++f) items.push_back({(int)i, f, ld.h_ptr[f + 1] - ld.h_ptr[f]});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.L > y.L; });
  std::vector<double> load(NX, 0.0);
  std::vector<int64_t> count(NX, 0);
  std::vector<std::vector<TileDesc>> bins(NX);
  for (const Item& it : items) {
    const lsx_plan* pl = b->pl[it.sys];
    const LayerDev& ld = pl->L[layer - 1];
    const int W = b->st[it.sys]->W;
    const int wt = (W == 1) ? 1 : (W + 16 * nb - 1) / (16 * nb);
    const int nrb = (it.L + 15) / 16;
    int x = 0;
    for (int y = 1; y < NX; ++y)
      if (count[y] < count[x] || (count[y] == count[x] && load[y] < load[x])) x = y;
    count[x] += (int64_t)nrb * wt;
    for (int rb = 0; rb < nrb; ++rb) {
      int32_t k0, k1;
      fibre_band(ld, it.f, rb, 1, k0, k1);
      load[x] += (double)wt * (std::min(k1, it.L) - k0 + 8);
      for (int wb = 0; wb < wt; ++wb) {
        TileDesc t;
        t.r0 = ld.h_ptr[it.f];
        t.L = it.L;
        t.rb = rb;
        t.wb = wb;
        t.poff = ld.h_poff[it.f];
        t.f = it.sys;
        t.d0 = ld.h_d0[it.f];
        t.k0 = k0;
        t.k1 = k1;
        t.bb = -1;
        t.pad_ = 0;
        bins[x].push_back(t);
      }
    }
  }
  TileDesc empty{};
  empty.f = -1;
  size_t maxlen = 0;
  for (auto& bn : bins) maxlen = std::max(maxlen, bn.size());
  out.clear();
  for (size_t i = 0; i < maxlen; ++i)
    for (int x = 0; x < NX; ++x) out.push_back(i < bins[x].size() ? bins[x][i] : empty);
  while (!out.empty() && out.back().f < 0) out.pop_back();
}

// Launches one batched pass; (cur, lay) follow the same rules as Runner.
static lsx_status batch_pass(lsx_batch* b, hipStream_t s, const PassSpec& p, int& cur, int& lay) {
  const int outlay = p.next;  // 0: canonical order
  const PatternKey k{p.layer, p.half, lay, outlay, p.phase_half, cur};
  const PassArgs* d = nullptr;
  bool gather = false;
  LSX_TRY(batch_args(b, k, &d, &gather));
  PassArgs a0{};
  a0.tiles = b->tiles[p.layer - 1].p;
  a0.in_pos = gather ? b->marker.p : nullptr;  // gather flag, uniform over the batch
  a0.batch = d;
  a0.persist = b->persist[p.layer - 1];
  a0.queue = b->queue.p;
  a0.u = b->u[p.layer - 1];
  LSX_HIP_TRY(launch_pass(s, b->fmt, b->w1 ? 1 : 2, b->ntiles[p.layer - 1], b->nb[p.layer - 1],
                          b->ks[p.layer - 1], a0, true));
  cur ^= 1;
  lay = outlay;
  return LSX_OK;
}

extern "C" lsx_status lsx_batch_create(lsx_plan* const* plans, lsx_state* const* states, int32_t n, lsx_batch** out) {
  if (!plans || !states || !out || n < 1) return fail(LSX_E_INVALID, "bad batch arguments");
  lsx_batch* b = new (std::nothrow) lsx_batch();
  if (!b) return fail(LSX_E_OOM, "host allocation failed");
  auto cleanup = [&](lsx_status e) {
    delete b;
    return e;
  };
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || !states[i] || states[i]->plan != plans[i])
      return cleanup(fail(LSX_E_STATE, "batch entry " + std::to_string(i) + ": state does not belong to plan"));
    if (plans[i]->scheme != plans[0]->scheme || plans[i]->fmt != plans[0]->fmt)
      return cleanup(fail(LSX_E_INVALID, "batch plans must share scheme and precision"));
    if (plans[i]->sys->nl != plans[0]->sys->nl)
      return cleanup(fail(LSX_E_INVALID, "batch systems must have the same number of layers"));
    if ((states[i]->W == 1) != (states[0]->W == 1))
      return cleanup(fail(LSX_E_INVALID, "batch states must be all W = 1 or all W >= 2"));
    for (int j = 0; j < i; ++j)
      if (states[j] == states[i]) return cleanup(fail(LSX_E_INVALID, "a state appears twice in the batch"));
    b->pl.push_back(plans[i]);
    b->st.push_back(states[i]);
  }
  b->fmt = plans[0]->fmt;
  b->scheme = plans[0]->scheme;
  b->nl = plans[0]->sys->nl;
  b->w1 = states[0]->W == 1;
  lsx_status e;
  if ((e = b->marker.alloc(1)) != LSX_OK) return cleanup(e);
  if ((e = b->queue.alloc(9)) != LSX_OK) return cleanup(e);
  if (hipMemset(b->queue.p, 0, 9 * sizeof(int32_t)) != hipSuccess)
    return cleanup(fail(LSX_E_HIP, "hipMemset of the tile queue failed"));
  // tile shape and launch mode: autotune over the combined tiles with the steady-state pass
  // patterns.  Modes: 0 one workgroup per tile (the hardware dispatcher balances), 2
  // persistent grid with a static stride, 1 persistent grid with per-XCD tile queues;
  // LSX_PERSIST forces one mode, LSX_NB / LSX_KS one shape.
  // u: groups of k-steps in flight per wave of the FP64 / FP32 tiles (0: two), as for states
  struct Shape {
    int nb, ks, pm, u;
  };
  std::vector<Shape> shapes;
  int maxW = 1;
  for (lsx_state* st : b->st) maxW = std::max(maxW, st->W);
  const bool tune_u = (b->fmt == PF_F64 || b->fmt == PF_F32) && std::getenv("LSX_PREFETCH") == nullptr;
  if (b->w1) {
    shapes.push_back({1, 4, 0, 0});
  } else {
    for (int nbv : {1, 2, 4})
      for (int k : {1, 2, 4})
        if (16 * nbv <= round_up(maxW, 16) && !(nbv == 4 && k == 4)) {
          shapes.push_back({nbv, k, 0, 0});
          if (tune_u) shapes.push_back({nbv, k, 0, 1});
        }
    const int fnb = env_int("LSX_NB", 0), fks = env_int("LSX_KS", 0);
    if (fnb > 0 || fks > 0) shapes.assign(1, Shape{fnb > 0 ? fnb : 1, fks > 0 ? fks : 2, 0, 0});
    else if (env_int("LSX_AUTOTUNE", 1) == 0) shapes.assign(1, Shape{1, 2, 0, 0});
  }
  const int fpm = env_int("LSX_PERSIST", -1);
  std::vector<int> modes = {0, 2, 1};
  if (fpm >= 0 && fpm <= 2) modes.assign(1, fpm);
  else if (env_int("LSX_AUTOTUNE", 1) == 0) modes.assign(1, 0);
  std::vector<Shape> cands;
  for (int m : modes)
    for (Shape c : shapes) {
      c.pm = m;
      cands.push_back(c);
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return cleanup(fail(LSX_E_HIP, "event creation failed"));
  }
  for (int layer = 1; layer <= b->nl; ++layer) {
    // time the first propagator slot the plans hold for this layer
    int slot = 0;
    while (slot < 2 && !b->pl[0]->L[layer - 1].prop[slot].present) ++slot;
    float best = -1.f;
    for (const Shape& c : cands) {
      std::vector<TileDesc> t;
      batch_tiles(b, layer, c.nb, t);
      DBuf<TileDesc> d;
      if ((e = d.upload(t, nullptr)) != LSX_OK) break;
      // time a steady-state pass (fibre-contiguous read, scattered write) into the work arrays
      std::swap(b->tiles[layer - 1].p, d.p);
      std::swap(b->tiles[layer - 1].n, d.n);
      const int save_nt = b->ntiles[layer - 1], save_nb = b->nb[layer - 1], save_ks = b->ks[layer - 1];
      const int save_pm = b->persist[layer - 1], save_u = b->u[layer - 1];
      b->ntiles[layer - 1] = (int)t.size();
      b->nb[layer - 1] = c.nb;
      b->ks[layer - 1] = c.ks;
      b->persist[layer - 1] = c.pm;
      b->u[layer - 1] = c.u;
      float ms = 0.f;
      if (cands.size() > 1) {
        int cur = 0, lay = layer;
        const PassSpec p{layer, slot, layer % b->nl + 1, -1};
        hipError_t he = hipSuccess;
        int c2 = 0, l2 = lay;
        if ((e = batch_pass(b, nullptr, p, c2, l2)) != LSX_OK) break;
        // five timed passes, then, for passes under 200 us, about 1 ms of them
        auto time_reps = [&](int reps, float& per) {
          float total = 0.f;
          he = hipEventRecord(e0, nullptr);
          for (int r = 0; r < reps && he == hipSuccess; ++r) {
            cur = 0;
            lay = layer;
            if ((e = batch_pass(b, nullptr, p, cur, lay)) != LSX_OK) return;
          }
          if (he == hipSuccess) he = hipEventRecord(e1, nullptr);
          if (he == hipSuccess) he = hipEventSynchronize(e1);
          if (he == hipSuccess) he = hipEventElapsedTime(&total, e0, e1);
          per = total / reps;
        };
        time_reps(5, ms);
        if (e == LSX_OK && he == hipSuccess && ms < 0.2f)
          time_reps(std::min(100, std::max(5, (int)(1.0f / std::max(ms, 1e-3f)))), ms);
        if (e != LSX_OK) break;
        if (he != hipSuccess) {
          e = fail(LSX_E_HIP, std::string("batch autotune: ") + hipGetErrorString(he));
          break;
        }
      }
      if (best < 0.f || ms < best) {
        best = ms;  // keep: the new tiles stay installed
      } else {
        // restore the previous best
        std::swap(b->tiles[layer - 1].p, d.p);
        std::swap(b->tiles[layer - 1].n, d.n);
        b->ntiles[layer - 1] = save_nt;
        b->nb[layer - 1] = save_nb;
        b->ks[layer - 1] = save_ks;
        b->persist[layer - 1] = save_pm;
        b->u[layer - 1] = save_u;
      }
    }
    if (e != LSX_OK) break;
    b->tuned_us[layer - 1] = cands.size() > 1 ? best * 1e3f : 0.f;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != LSX_OK) return cleanup(e);
  for (int layer = 1; layer <= b->nl; ++layer)
    if (b->persist[layer - 1])
      for (const int32_t* gather : {static_cast<const int32_t*>(nullptr), static_cast<const int32_t*>(b->marker.p)}) {
        PassArgs a0{};
        a0.in_pos = gather;
        a0.persist = b->persist[layer - 1];
        a0.queue = b->queue.p;
        a0.u = b->u[layer - 1];
        if (prepare_persistent(b->fmt, b->w1 ? 1 : 2, b->nb[layer - 1], b->ks[layer - 1], a0) != hipSuccess)
          return cleanup(fail(LSX_E_HIP, "persistent launch setup failed"));
      }
  if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(LSX_E_HIP, "batch setup failed"));
  for (lsx_state* st : b->st) st->nbatches++;
  for (lsx_state* st : b->st) b->bufs.emplace_back(st->buf[0], st->buf[1]);
  *out = b;
  return LSX_OK;
}

extern "C" lsx_status lsx_batch_step(lsx_batch* b, int64_t nsteps, void* stream) {
  if (!b) return fail(LSX_E_INVALID, "null batch");
  if (nsteps < 0) return fail(LSX_E_INVALID, "nsteps must be >= 0");
  if (nsteps == 0) return LSX_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // argument arrays refer to the states' arrays: rebuild them if a state swapped its arrays
  for (size_t i = 0; i < b->st.size(); ++i)
    if (b->bufs[i].first != b->st[i]->buf[0] || b->bufs[i].second != b->st[i]->buf[1]) {
      b->args.clear();
      batch_drop_graph(b);
      for (size_t j = 0; j < b->st.size(); ++j) b->bufs[j] = {b->st[j]->buf[0], b->st[j]->buf[1]};
      break;
    }
  std::vector<PassSpec> head, body, tail;
  int64_t reps = 0;
  step_sequence(b->scheme, b->nl, nsteps, head, body, tail, reps);
  int cur = 0, lay = 0;  // canonical order
  for (const PassSpec& p : head) LSX_TRY(batch_pass(b, s, p, cur, lay));
  // The captured body must return to the (array, layout) state it starts from, so a body with
  // an odd number of passes (three-layer Lie) is captured twice over; an odd repetition left
  // over runs eagerly after the replays.
  std::vector<PassSpec> gbody = body;
  int64_t greps = reps, extra = 0;
  if (body.size() % 2 == 1) {
    gbody.insert(gbody.end(), body.begin(), body.end());
    greps = reps / 2;
    extra = reps % 2;
  }
  // one graph holds kb repetitions of the (even) body, about kGraphPasses passes; the
  // repetitions short of a whole graph run eagerly
  const int64_t kb = std::max<int64_t>(1, graph_passes(kBatchGraphPasses) / std::max<int64_t>(1, (int64_t)gbody.size()));
  const bool use_graph = use_step_graphs(b->tuned_us, b->nl) && !gbody.empty() && greps >= kb;
  int64_t eager = use_graph ? greps % kb : greps;
  if (use_graph) {
    // the body returns to the same (array, layout) state, so one captured graph serves
    // every repetition; it is built on first use and kept with the batch
    const int cur0 = cur, lay0 = lay;
    if (b->exec && b->graph_k != kb) batch_drop_graph(b);
    if (!b->exec) {
      {
        // build every argument array first: capture must not do synchronous copies
        int c2 = cur, l2 = lay;
        for (const PassSpec& p : gbody) {
          const int outlay = p.next;
          const PassArgs* d = nullptr;
          LSX_TRY(batch_args(b, PatternKey{p.layer, p.half, l2, outlay, p.phase_half, c2}, &d));
          c2 ^= 1;
          l2 = outlay;
        }
        if (!b->cap) LSX_HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        LSX_HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        lsx_status cap_err = LSX_OK;
        for (int64_t i = 0; i < kb && cap_err == LSX_OK; ++i)
          for (const PassSpec& p : gbody)
            if ((cap_err = batch_pass(b, b->cap, p, cur, lay)) != LSX_OK) break;
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(b->cap, &g);
        if (cap_err != LSX_OK) {
          if (g) (void)hipGraphDestroy(g);
          return cap_err;
        }
        LSX_HIP_TRY(ee);
        b->graph = g;
        LSX_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_k = kb;
        cur = cur0;
        lay = lay0;
      }
    }
    for (int64_t r = 0; r < greps / kb; ++r) LSX_HIP_TRY(hipGraphLaunch(b->exec, s));
    // the captured body has an even number of passes and ends in the layout it started from
    cur = cur0;
    lay = lay0;
  }
  for (int64_t r = 0; r < eager; ++r)
    for (const PassSpec& p : gbody) LSX_TRY(batch_pass(b, s, p, cur, lay));
  for (int64_t r = 0; r < extra; ++r)
    for (const PassSpec& p : body) LSX_TRY(batch_pass(b, s, p, cur, lay));
  for (const PassSpec& p : tail) LSX_TRY(batch_pass(b, s, p, cur, lay));
  if (cur != 0) {
    for (lsx_state* st : b->st)
      LSX_HIP_TRY(hipMemcpyAsync(st->buf[0], st->buf[1], (size_t)st->plan->sys->N * st->W * sizeof(double2),
                                 hipMemcpyDeviceToDevice, s));
  }
  return LSX_OK;
}

extern "C" lsx_status lsx_batch_tuning(const lsx_batch* b, int32_t layer, int32_t* nb, int32_t* ks, double* pass_us,
                                       int32_t* launch_mode) {
  if (!b) return fail(LSX_E_INVALID, "null batch");
  if (layer < 1 || layer > b->nl) return fail(LSX_E_INVALID, "layer out of range");
  if (launch_mode) *launch_mode = b->persist[layer - 1];
  if (nb) *nb = b->nb[layer - 1];
  if (ks) *ks = b->ks[layer - 1];
  if (pass_us) *pass_us = b->tuned_us[layer - 1];
  return LSX_OK;
}

extern "C" lsx_status lsx_batch_destroy(lsx_batch* b) {
  if (!b) return LSX_OK;
  for (lsx_state* st : b->st) st->nbatches--;
  delete b;
  return LSX_OK;
}

// ================================================================ proposal network
struct lsx_mlp {
  int nin = 0, n = 0;
  DBuf<float> theta, m, v, grad, partial, z, dz;
  DBuf<double> lg, out;
  DBuf<int32_t> active;
  int64_t t = 0;  // Adam steps taken
  int nsamplers = 0;
};

template <typename T>
static lsx_status ensure(DBuf<T>& b, size_t n) {
  if (b.n >= n && b.p) return LSX_OK;
  return b.alloc(n);
}

extern "C" lsx_status lsx_mlp_create(int32_t nin, lsx_mlp** out) {
  if (!out) return fail(LSX_E_INVALID, "null argument");
  if (nin < 1 || nin > 8) return fail(LSX_E_INVALID, "nin must be in [1, 8]");
  std::unique_ptr<lsx_mlp> m(new (std::nothrow) lsx_mlp());
  if (!m) return fail(LSX_E_OOM, "host allocation failed");
  m->nin = nin;
  m->n = mlp_nparams(nin);
  LSX_TRY(m->theta.alloc(m->n));
  LSX_TRY(m->m.alloc(m->n));
  LSX_TRY(m->v.alloc(m->n));
  LSX_TRY(m->grad.alloc(m->n));
  LSX_TRY(m->out.alloc(2));
  LSX_HIP_TRY(hipMemset(m->theta.p, 0, m->n * sizeof(float)));
  LSX_HIP_TRY(hipMemset(m->m.p, 0, m->n * sizeof(float)));
  LSX_HIP_TRY(hipMemset(m->v.p, 0, m->n * sizeof(float)));
  *out = m.release();
  return LSX_OK;
}

extern "C" lsx_status lsx_mlp_nparams(const lsx_mlp* m, int64_t* n) {
  if (!m || !n) return fail(LSX_E_INVALID, "null argument");
  *n = m->n;
  return LSX_OK;
}

extern "C" lsx_status lsx_mlp_set(lsx_mlp* m, const float* theta, void* stream) {
  if (!m || !theta) return fail(LSX_E_INVALID, "null argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  LSX_HIP_TRY(hipMemcpyAsync(m->theta.p, theta, m->n * sizeof(float), hipMemcpyHostToDevice, s));
  LSX_HIP_TRY(hipMemsetAsync(m->m.p, 0, m->n * sizeof(float), s));
  LSX_HIP_TRY(hipMemsetAsync(m->v.p, 0, m->n * sizeof(float), s));
  LSX_HIP_TRY(hipStreamSynchronize(s));
  m->t = 0;
  return LSX_OK;
}

extern "C" lsx_status lsx_mlp_get(const lsx_mlp* m, float* theta, void* stream) {
  if (!m || !theta) return fail(LSX_E_INVALID, "null argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  LSX_HIP_TRY(hipMemcpyAsync(theta, m->theta.p, m->n * sizeof(float), hipMemcpyDeviceToHost, s));
  LSX_HIP_TRY(hipStreamSynchronize(s));
  return LSX_OK;
}

extern "C" lsx_status lsx_mlp_forward(const lsx_mlp* m, const float* X, int64_t M, float* z, void* stream) {
  if (!m || (M > 0 && (!X || !z))) return fail(LSX_E_INVALID, "null argument");
  if (M < 0) return fail(LSX_E_INVALID, "M must be >= 0");
  LSX_HIP_TRY(launch_mlp_fwd(reinterpret_cast<hipStream_t>(stream), m->theta.p, m->nin, X, M, z));
  return LSX_OK;
}

static lsx_status mlp_backward(lsx_mlp* m, const float* X, int64_t M, const float* dz, const double* gscale,
                               float* grad, hipStream_t s) {
  LSX_TRY(ensure(m->partial, (size_t)mlp_bwd_blocks(M) * m->n));
  LSX_HIP_TRY(launch_mlp_bwd(s, m->theta.p, m->nin, X, M, dz, gscale, m->partial.p, grad));
  return LSX_OK;
}

extern "C" lsx_status lsx_mlp_backward(lsx_mlp* m, const float* X, int64_t M, const float* dz, float* grad,
                                       void* stream) {
  if (!m || !grad || (M > 0 && (!X || !dz))) return fail(LSX_E_INVALID, "null argument");
  if (M < 0) return fail(LSX_E_INVALID, "M must be >= 0");
  return mlp_backward(m, X, M, dz, nullptr, grad, reinterpret_cast<hipStream_t>(stream));
}

static lsx_status mlp_loss(lsx_mlp* m, const float* z, const double* b, const int64_t* gptr, int64_t G, double eps,
                           double* out, float* dz, hipStream_t s) {
  LSX_TRY(ensure(m->lg, (size_t)std::max<int64_t>(G, 1)));
  LSX_TRY(ensure(m->active, (size_t)std::max<int64_t>(G, 1)));
  LSX_HIP_TRY(launch_loss(s, z, b, gptr, G, eps, m->lg.p, m->active.p, dz, out));
  return LSX_OK;
}

extern "C" lsx_status lsx_mlp_loss(lsx_mlp* m, const float* z, const double* b, const int64_t* gptr,
                                   int64_t ngroups, double eps, double* out, float* dz, void* stream) {
  if (!m || !out || (ngroups > 0 && (!z || !b || !gptr || !dz))) return fail(LSX_E_INVALID, "null argument");
  if (ngroups < 0) return fail(LSX_E_INVALID, "ngroups must be >= 0");
  if (!(eps >= 0.0 && eps <= 1.0)) return fail(LSX_E_INVALID, "eps must be in [0, 1]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (ngroups == 0) {
    LSX_HIP_TRY(hipMemsetAsync(out, 0, 2 * sizeof(double), s));
    return LSX_OK;
  }
  LSX_TRY(mlp_loss(m, z, b, gptr, ngroups, eps, out, dz, s));
  // dz of the mean: scale by 1 / (number of active groups), read from out[1]
  int64_t M = 0;
  LSX_HIP_TRY(hipMemcpyAsync(&M, gptr + ngroups, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LSX_HIP_TRY(hipStreamSynchronize(s));
  LSX_HIP_TRY(launch_scale_f32(s, M, out + 1, dz));
  return LSX_OK;
}

static lsx_status mlp_adam(lsx_mlp* m, const float* grad, double lr, double b1, double b2, double eps,
                           hipStream_t s) {
  m->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow(b1, (double)m->t));
  const double c2 = 1.0 / (1.0 - std::pow(b2, (double)m->t));
  LSX_HIP_TRY(launch_adam(s, m->n, m->theta.p, m->m.p, m->v.p, grad, lr, b1, b2, eps, c1, c2));
  return LSX_OK;
}

static bool adam_args_ok(double lr, double b1, double b2, double eps) {
  return std::isfinite(lr) && b1 >= 0.0 && b1 < 1.0 && b2 >= 0.0 && b2 < 1.0 && eps > 0.0;
}

extern "C" lsx_status lsx_mlp_adam(lsx_mlp* m, const float* grad, double lr, double b1, double b2, double eps,
                                   void* stream) {
  if (!m || !grad) return fail(LSX_E_INVALID, "null argument");
  if (!adam_args_ok(lr, b1, b2, eps)) return fail(LSX_E_INVALID, "bad Adam hyper-parameters");
  return mlp_adam(m, grad, lr, b1, b2, eps, reinterpret_cast<hipStream_t>(stream));
}

extern "C" lsx_status lsx_mlp_train_step(lsx_mlp* m, const float* X, int64_t M, const double* b,
                                         const int64_t* gptr, int64_t ngroups, double eps, double lr, double b1,
                                         double b2, double adam_eps, double* out, void* stream) {
  if (!m || !X || !b || !gptr || !out) return fail(LSX_E_INVALID, "null argument");
  if (M < 1 || ngroups < 1) return fail(LSX_E_INVALID, "need M >= 1 rows and ngroups >= 1");
  if (!(eps >= 0.0 && eps <= 1.0)) return fail(LSX_E_INVALID, "eps must be in [0, 1]");
  if (!adam_args_ok(lr, b1, b2, adam_eps)) return fail(LSX_E_INVALID, "bad Adam hyper-parameters");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  LSX_TRY(ensure(m->z, (size_t)M));
  LSX_TRY(ensure(m->dz, (size_t)M));
  LSX_HIP_TRY(launch_mlp_fwd(s, m->theta.p, m->nin, X, M, m->z.p));
  LSX_TRY(mlp_loss(m, m->z.p, b, gptr, ngroups, eps, out, m->dz.p, s));
  LSX_TRY(mlp_backward(m, X, M, m->dz.p, out + 1, m->grad.p, s));
  return mlp_adam(m, m->grad.p, lr, b1, b2, adam_eps, s);
}

extern "C" lsx_status lsx_mlp_destroy(lsx_mlp* m) {
  if (!m) return LSX_OK;
  if (m->nsamplers > 0) return fail(LSX_E_STATE, "network is attached to a sampler");
  delete m;
  return LSX_OK;
}

// ================================================================ stochastic steps
// Sampled fibre sub-steps run in the canonical layout.  After the draws, every fibre gets
// the list of columns (wavepackets) that drew it; tiles cover only those (fibre, column)
// pairs, so the pass does the method's own work rather than a full pass.  The weighted
// pass reads the state and writes the sampled (rows, columns) into the work array, from
// which they are copied back; every other entry is left untouched.  The tile lists are
// built on the device, with no host round trip.
static constexpr int kSamplerMaxFibres = 2048;

struct lsx_sampler {
  lsx_plan* pl = nullptr;
  lsx_state* st = nullptr;
  lsx_mlp* mlp = nullptr;
  int p[2] = {0, 0};
  double eps = 0.0;
  int nf[2] = {0, 0};
  int ntiles[2] = {0, 0};  // tiles of a pass over every fibre and column: the launch bound
  DBuf<TileDesc> tiles[2];  // tiles of the sampled (fibre, column) pairs, built per sub-step
  DBuf<int32_t> cols[2], ncols[2], off[2], fid[2], d0[2];
  DBuf<int64_t> poff[2];
  // band of every (fibre, 16-row block): [2 (bptr[f] + rb)] = k0, [.. + 1] = k1 (fibre positions)
  DBuf<int32_t> bptr[2], band[2];
  DBuf<int32_t> count;
  DBuf<double> wt[2], mass, sfeat[2];
  DBuf<float> X, z;
};

// column block of the sampled passes: one 16-column block per tile (the sampled columns of
// a fibre are typically few)
static constexpr int kSampledNB = 1;

extern "C" lsx_status lsx_sampler_create(lsx_plan* pl, lsx_state* st, int32_t p1, int32_t p2, double eps,
                                         lsx_sampler** out) {
  LSX_TRY(check_pair(pl, st));
  if (!out) return fail(LSX_E_INVALID, "null argument");
  if (p1 < 0 || p2 < 0) return fail(LSX_E_INVALID, "p1, p2 must be >= 0");
  if (!(eps >= 0.0 && eps <= 1.0)) return fail(LSX_E_INVALID, "eps must be in [0, 1]");
  const lsx_system* sys = pl->sys;
  if (sys->nl != 2 || !sys->standard) return fail(LSX_E_INVALID, "samplers hold two-layer systems built from lattices");
  const int W = st->W, d = sys->d;
  for (int j = 0; j < 2; ++j)
    if (pl->L[j].nf > kSamplerMaxFibres)
      return fail(LSX_E_INVALID, "sampler supports at most 2048 fibres per layer");
  std::unique_ptr<lsx_sampler> sm(new (std::nothrow) lsx_sampler());
  if (!sm) return fail(LSX_E_OOM, "host allocation failed");
  sm->pl = pl;
  sm->st = st;
  sm->p[0] = p1;
  sm->p[1] = p2;
  sm->eps = eps;
  const double kmax = std::sqrt(2.0 * sys->Ec);
  int maxnf = 1;
  for (int j = 0; j < 2; ++j) {
    const LayerDev& ld = pl->L[j];
    const FibreTable& ft = sys->fib[j];
    const int nf = ld.nf;
    sm->nf[j] = nf;
    maxnf = std::max(maxnf, nf);
    const int nwb = (W + 16 * kSampledNB - 1) / (16 * kSampledNB);
    int64_t ntiles = 0;
    for (int f = 0; f < nf; ++f) ntiles += (int64_t)((ld.h_ptr[f + 1] - ld.h_ptr[f] + 15) / 16) * nwb;
    if (ntiles > INT32_MAX) return fail(LSX_E_INVALID, "too many tiles for one sampled pass");
    sm->ntiles[j] = (int)ntiles;
    LSX_TRY(sm->tiles[j].alloc((size_t)std::max<int64_t>(ntiles, 1)));
    LSX_TRY(sm->cols[j].alloc((size_t)std::max(nf, 1) * W));
    LSX_TRY(sm->ncols[j].alloc(std::max(nf, 1)));
    LSX_TRY(sm->off[j].alloc(std::max(nf, 1)));
    std::vector<int64_t> poff(nf, 0);
    std::vector<int32_t> d0(nf, 0);
    for (int f = 0; f < nf; ++f) {
      poff[f] = ld.h_poff.empty() ? 0 : ld.h_poff[f];
      d0[f] = ld.h_d0.empty() ? ld.h_ptr[f] : ld.h_d0[f];
    }
    LSX_TRY(sm->poff[j].upload(poff, nullptr));
    LSX_TRY(sm->d0[j].upload(d0, nullptr));
    {
      std::vector<int32_t> bp(std::max(nf, 1), 0), bd;
      for (int f = 0; f < nf; ++f) {
        bp[f] = (int32_t)(bd.size() / 2);
        for (int rb = 0; rb < (ld.h_ptr[f + 1] - ld.h_ptr[f] + 15) / 16; ++rb) {
          int32_t k0, k1;
          fibre_band(ld, f, rb, 1, k0, k1);
          bd.push_back(k0);
          bd.push_back(k1);
        }
      }
      if (bd.empty()) bd.assign(2, 0);
      LSX_TRY(sm->bptr[j].upload(bp, nullptr));
      LSX_TRY(sm->band[j].upload(bd, nullptr));
    }
    // fibre of every canonical row, and the per-fibre shift features
    std::vector<int32_t> fid((size_t)sys->N, 0);
    std::vector<double> sf((size_t)nf * (d + 1), 0.0);
    const double* B = sys->B[j == 0 ? 1 : 0];  // layer-1 fibres are shifted by G2 n, layer-2 by G1 m
    const int other = (j == 0) ? d : 0;       // offset of the fibre's fixed index inside (m, n)
    for (int f = 0; f < nf; ++f) {
      for (int a = ft.ptr[f]; a < ft.ptr[f + 1]; ++a) fid[ft.rows[a]] = f;
      if (ft.ptr[f + 1] > ft.ptr[f]) {
        const int32_t* mn = &sys->mn[(size_t)ft.rows[ft.ptr[f]] * 2 * d];
        double s2 = 0.0;
        for (int k = 0; k < d; ++k) {
          double g = 0.0;
          for (int l = 0; l < d; ++l) g += B[k * d + l] * mn[other + l];
          const double x = g / kmax;
          sf[(size_t)f * (d + 1) + k] = x;
          s2 += x * x;
        }
        sf[(size_t)f * (d + 1) + d] = s2;
      }
    }
    LSX_TRY(sm->fid[j].upload(fid, nullptr));
    LSX_TRY(sm->sfeat[j].upload(sf, nullptr));
    LSX_TRY(sm->wt[j].alloc((size_t)std::max(nf, 1) * W));
  }
  LSX_TRY(sm->count.alloc(2));
  LSX_TRY(sm->mass.alloc((size_t)maxnf * W));
  LSX_TRY(sm->X.alloc((size_t)maxnf * W * (d + 3)));
  LSX_TRY(sm->z.alloc((size_t)maxnf * W));
  LSX_HIP_TRY(hipDeviceSynchronize());
  st->nsamplers++;
  *out = sm.release();
  return LSX_OK;
}

extern "C" lsx_status lsx_sampler_set_mlp(lsx_sampler* sm, lsx_mlp* mlp) {
  if (!sm) return fail(LSX_E_INVALID, "null argument");
  if (mlp && mlp->nin != sm->pl->sys->d + 3) return fail(LSX_E_INVALID, "network must take d + 3 inputs");
  if (sm->mlp) sm->mlp->nsamplers--;
  sm->mlp = mlp;
  if (mlp) mlp->nsamplers++;
  return LSX_OK;
}

extern "C" lsx_status lsx_sampler_destroy(lsx_sampler* sm) {
  if (!sm) return LSX_OK;
  if (sm->mlp) sm->mlp->nsamplers--;
  sm->st->nsamplers--;
  delete sm;
  return LSX_OK;
}

namespace {
// canonical-layout position table of a layer's fibre positions (null: identity)
const int32_t* canon_pos(const lsx_plan* pl, int layer) { return layout_map(pl, layer, 0); }

PassArgs canon_pass_args(const lsx_plan* pl, const lsx_state* st, int layer, int half) {
  const LayerDev& ld = pl->L[layer - 1];
  PassArgs a;
  a.in_pos = canon_pos(pl, layer);
  a.out_pos = canon_pos(pl, layer);
  a.P = ld.prop[half].data.p;
  a.diag = pl->diag.p ? pl->diag.p + (size_t)((layer - 1) * 3 + half) * pl->sys->N : nullptr;
  a.X = st->buf[0];
  a.Y = st->buf[1];
  a.zero = pl->zero.p;
  a.orbit = ld.d_orbit.p;
  a.orbit_max = ld.orbit_max;
  a.W = st->W;
  return a;
}

// state's current coefficients -> network inputs of `layer` in sm->X
lsx_status sampler_features(lsx_sampler* sm, int layer, float* X, hipStream_t s) {
  const lsx_plan* pl = sm->pl;
  const LayerDev& ld = pl->L[layer - 1];
  const int W = sm->st->W;
  LSX_HIP_TRY(launch_fibre_mass(s, ld.nf, ld.ptr.p, ld.rows.p, W, sm->st->buf[0], sm->mass.p));
  LSX_HIP_TRY(launch_features(s, ld.nf, W, pl->sys->d, sm->sfeat[layer - 1].p, sm->mass.p,
                              layer == 1 ? -1.f : 1.f, X));
  return LSX_OK;
}

// one sampled sub-step of `layer` with propagators `half`, uniforms u [W][ustride]
lsx_status sampled_substep(lsx_sampler* sm, int layer, int half, const double* u, int ustride, hipStream_t s) {
  lsx_plan* pl = sm->pl;
  lsx_state* st = sm->st;
  const int j = layer - 1;
  const int W = st->W, nf = sm->nf[j];
  if (nf == 0) return LSX_OK;
  if (!pl->L[j].prop[half].present) return fail(LSX_E_INVALID, "plan holds no propagator for this sub-step");
  if (sm->p[j] == 0) {  // fallback: the deterministic pass
    Runner r{pl, st, s};
    LSX_TRY(r.pass(layer, half, 0, -1));
    return r.finish();
  }
  const float* z = nullptr;
  if (sm->mlp) {
    LSX_TRY(sampler_features(sm, layer, sm->X.p, s));
    LSX_HIP_TRY(launch_mlp_fwd(s, sm->mlp->theta.p, sm->mlp->nin, sm->X.p, (int64_t)W * nf, sm->z.p));
    z = sm->z.p;
  }
  LSX_HIP_TRY(launch_sample_weights(s, nf, W, sm->p[j], ustride, u, z, sm->eps, sm->wt[j].p));
  const LayerDev& ld = pl->L[j];
  LSX_HIP_TRY(launch_sampled_tiles(s, nf, W, kSampledNB, sm->wt[j].p, ld.ptr.p, sm->poff[j].p, sm->d0[j].p,
                                   sm->bptr[j].p, sm->band[j].p, sm->cols[j].p, sm->ncols[j].p, sm->off[j].p,
                                   sm->tiles[j].p, sm->count.p + j));
  PassArgs a = canon_pass_args(pl, st, layer, half);
  a.tiles = sm->tiles[j].p;
  a.tcount = sm->count.p + j;
  a.wt = sm->wt[j].p;
  a.cols = sm->cols[j].p;
  a.ncols = sm->ncols[j].p;
  // sampled tiles are per row block: a fibre-length split, never the row-split kernel
  LSX_HIP_TRY(launch_pass(s, pl->fmt, W, sm->ntiles[j], kSampledNB, st->ks[j] > 0 ? st->ks[j] : 2, a));
  LSX_HIP_TRY(launch_copy_cols(s, sm->ntiles[j], sm->tiles[j].p, sm->count.p + j, kSampledNB, canon_pos(pl, layer),
                               W, sm->cols[j].p, sm->ncols[j].p, st->buf[1], st->buf[0]));
  return LSX_OK;
}

lsx_status phase_canon(lsx_plan* pl, lsx_state* st, int half, hipStream_t s) {
  if (pl->kappa == 0.0 || pl->sys->N == 0) return LSX_OK;
  if (!pl->phase[half].p) return fail(LSX_E_INVALID, "plan holds no phase table for this slot");
  LSX_HIP_TRY(launch_phase_apply(s, pl->sys->N, st->W, pl->phase[half].p, st->buf[0]));
  return LSX_OK;
}

// Alg. 1 / Alg. 4 step from buf[0] into buf[1], then back into buf[0]
lsx_status si_once(lsx_plan* pl, lsx_state* st, const double* wt1, const int32_t* fid1, const double* wt2,
                   const int32_t* fid2, hipStream_t s) {
  const lsx_system* sys = pl->sys;
  LSX_HIP_TRY(launch_si_step(s, sys->N, st->W, pl->tau, pl->K2.p, sys->pot[0].nv, pl->L[0].nbr.p, pl->L[0].v.p,
                             wt1, fid1, sys->pot[1].nv, pl->L[1].nbr.p, pl->L[1].v.p, wt2, fid2, st->buf[0],
                             st->buf[1], pl->zero.p));
  Runner r{pl, st, s};
  r.cur = 1;
  return r.finish();
}
}  // namespace

extern "C" lsx_status lsx_si_step(lsx_plan* pl, lsx_state* st, int64_t nsteps, void* stream) {
  LSX_TRY(check_pair(pl, st));
  if (nsteps < 0) return fail(LSX_E_INVALID, "nsteps must be >= 0");
  if (pl->sys->nl != 2 || !pl->sys->standard)
    return fail(LSX_E_INVALID, "the semi-implicit step takes two-layer systems built from lattices");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int64_t k = 0; k < nsteps && pl->sys->N > 0; ++k) LSX_TRY(si_once(pl, st, nullptr, nullptr, nullptr, nullptr, s));
  return LSX_OK;
}

extern "C" lsx_status lsx_rb_step(lsx_sampler* sm, const double* u, int64_t nsteps, void* stream) {
  if (!sm) return fail(LSX_E_INVALID, "null argument");
  if (nsteps < 0) return fail(LSX_E_INVALID, "nsteps must be >= 0");
  if (nsteps == 0 || sm->pl->sys->N == 0) return LSX_OK;
  if (!u) return fail(LSX_E_INVALID, "null uniforms");
  for (int j = 0; j < 2; ++j)
    if (sm->p[j] < 1 || sm->p[j] > sm->nf[j]) return fail(LSX_E_INVALID, "random batch needs 1 <= p_j <= nfibres_j");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int W = sm->st->W, pmax = std::max(sm->p[0], sm->p[1]);
  const int64_t per = (int64_t)W * pmax;
  for (int64_t k = 0; k < nsteps; ++k) {
    for (int j = 0; j < 2; ++j)
      LSX_HIP_TRY(launch_subset_weights(s, sm->nf[j], W, sm->p[j], pmax, u + (2 * k + j) * per, sm->wt[j].p));
    LSX_TRY(si_once(sm->pl, sm->st, sm->wt[0].p, sm->fid[0].p, sm->wt[1].p, sm->fid[1].p, s));
  }
  return LSX_OK;
}

extern "C" lsx_status lsx_ss_step(lsx_sampler* sm, const double* u, int64_t nsteps, void* stream) {
  if (!sm) return fail(LSX_E_INVALID, "null argument");
  if (nsteps < 0) return fail(LSX_E_INVALID, "nsteps must be >= 0");
  if (nsteps == 0 || sm->pl->sys->N == 0) return LSX_OK;
  if (!u && (sm->p[0] > 0 || sm->p[1] > 0)) return fail(LSX_E_INVALID, "null uniforms");
  lsx_plan* pl = sm->pl;
  if (pl->scheme == LSX_YOSHIDA4) return fail(LSX_E_INVALID, "stochastic steps take Lie or Strang schemes");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool strang = scheme_strang(pl->scheme);
  // (layer, propagator half, phase half after it or -1)
  struct Sub {
    int layer, half, ph;
  };
  const Sub lie[2] = {{1, 0, 0}, {2, 0, -1}};
  const Sub str[3] = {{1, 1, 1}, {2, 0, 1}, {1, 1, -1}};
  const Sub* subs = strang ? str : lie;
  const int nsub = strang ? 3 : 2;
  const int W = sm->st->W, pmax = std::max(1, std::max(sm->p[0], sm->p[1]));
  const int64_t per = (int64_t)W * pmax;
  for (int64_t k = 0; k < nsteps; ++k)
    for (int i = 0; i < nsub; ++i) {
      const double* uk = u ? u + (k * nsub + i) * per : nullptr;
      LSX_TRY(sampled_substep(sm, subs[i].layer, subs[i].half, uk, pmax, s));
      if (subs[i].ph >= 0) LSX_TRY(phase_canon(pl, sm->st, subs[i].ph, s));
    }
  return LSX_OK;
}

extern "C" lsx_status lsx_sampler_weights(lsx_sampler* sm, int32_t layer, int32_t mode, const float* z,
                                          const double* u, double* wt, void* stream) {
  if (!sm || !u || !wt) return fail(LSX_E_INVALID, "null argument");
  if (layer != 1 && layer != 2) return fail(LSX_E_INVALID, "layer must be 1 or 2");
  const int j = layer - 1, p = sm->p[j], nf = sm->nf[j];
  if (p < 1) return fail(LSX_E_INVALID, "p of this layer must be >= 1");
  if (nf == 0) return LSX_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (mode == 0) {
    LSX_HIP_TRY(launch_sample_weights(s, nf, sm->st->W, p, p, u, z, sm->eps, wt));
  } else if (mode == 1) {
    if (p > nf) return fail(LSX_E_INVALID, "subsets need p <= nfibres");
    LSX_HIP_TRY(launch_subset_weights(s, nf, sm->st->W, p, p, u, wt));
  } else {
    return fail(LSX_E_INVALID, "mode must be 0 or 1");
  }
  return LSX_OK;
}

extern "C" lsx_status lsx_sampler_features(lsx_sampler* sm, int32_t layer, float* X, void* stream) {
  if (!sm || !X) return fail(LSX_E_INVALID, "null argument");
  if (layer != 1 && layer != 2) return fail(LSX_E_INVALID, "layer must be 1 or 2");
  if (sm->nf[layer - 1] == 0) return LSX_OK;
  return sampler_features(sm, layer, X, reinterpret_cast<hipStream_t>(stream));
}

extern "C" lsx_status lsx_sampler_increments(lsx_sampler* sm, int32_t layer, int32_t half, double* b,
                                             void* stream) {
  if (!sm || !b) return fail(LSX_E_INVALID, "null argument");
  if (layer != 1 && layer != 2) return fail(LSX_E_INVALID, "layer must be 1 or 2");
  if (half < 0 || half > 2) return fail(LSX_E_INVALID, "slot must be 0, 1 or 2");
  lsx_plan* pl = sm->pl;
  lsx_state* st = sm->st;
  const LayerDev& ld = pl->L[layer - 1];
  if (ld.nf == 0) return LSX_OK;
  if (!ld.prop[half].present) return fail(LSX_E_INVALID, "plan holds no propagator for this layer/half");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  PassArgs a = canon_pass_args(pl, st, layer, half);
  a.tiles = st->tiles[layer - 1].p;
  LSX_HIP_TRY(launch_pass(s, pl->fmt, st->W, st->ntiles[layer - 1], st->nb[layer - 1], st->ks[layer - 1], a));
  LSX_HIP_TRY(launch_fibre_incr(s, ld.nf, ld.ptr.p, ld.rows.p, st->W, st->buf[0], st->buf[1], b));
  return LSX_OK;
}

// Block structure of U(1) tensors and the tensor part of the C ABI.
//
// A block is a tuple of sector indices whose flux (incoming charges minus
// outgoing charges) vanishes (Sec. "UniTensor with Symmetries"); blocks are
// kept in lexicographic order of the tuple with leg 0 most significant,
// which is the order the paper prints for its rank-3 example (Sec.
// "Symmetric UniTensor").  Each block is a row-major array and the blocks
// follow each other in one flat buffer.
#include <algorithm>
#include <cstring>
#include <stdexcept>

#include "plan.h"

namespace bst {

static thread_local std::string g_last_error;

void fail(bst_status s, const std::string& msg) { throw Error{s, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(BST_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static std::string key_of(const int32_t* t, int rank) {
  return std::string(reinterpret_cast<const char*>(t), sizeof(int32_t) * (size_t)rank);
}

void TensorDesc::build() {
  const int r = rank();
  qn.clear();
  shape.clear();
  offset.clear();
  lookup.clear();
  // Per-suffix reachable flux range of the first charge component, to prune
  // the lexicographic walk (U(1) only; a Z_n flux wraps, so no pruning).
  const int nsym = r > 0 ? legs[0].nsym() : 1;
  const bool prune = r > 0 && legs[0].modulus(0) == 0;
  std::vector<int64_t> lo(r + 1, 0), hi(r + 1, 0);
  for (int i = r - 1; i >= 0; --i) {
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (int32_t q : legs[i].q) {
      int64_t f = (int64_t)legs[i].dir * q;
      mn = std::min(mn, f);
      mx = std::max(mx, f);
    }
    lo[i] = lo[i + 1] + mn;
    hi[i] = hi[i + 1] + mx;
  }
  // A component's total flux vanishes: exactly for U(1), modulo n for Z_n
  // (the combine rule adds charges, the reverse rule negates them on
  // outgoing legs).
  auto vanishes = [](int64_t f, int32_t n) { return n == 0 ? f == 0 : f % n == 0; };
  std::vector<int32_t> t(r, 0);
  int64_t off = 0;
  // Iterative depth-first walk in lexicographic order.
  std::vector<int64_t> flux(r + 1, 0);
  int depth = 0;
  if (r == 0) {
    offset.push_back(0);
    lookup[key_of(t.data(), 0)] = 0;
    nblocks = 1;
    numel = 1;
    return;
  }
  t[0] = -1;
  while (depth >= 0) {
    t[depth]++;
    if (t[depth] >= (int32_t)legs[depth].q.size()) {
      depth--;
      continue;
    }
    int64_t f = flux[depth] + (int64_t)legs[depth].dir * legs[depth].q[t[depth]];
    // remaining legs must be able to cancel f
    if (prune && (f + lo[depth + 1] > 0 || f + hi[depth + 1] < 0)) continue;
    if (depth == r - 1) {
      if (!vanishes(f, legs[0].modulus(0))) continue;
      bool ok = true;
      for (int c = 1; c < nsym && ok; ++c) {
        int64_t fc = 0;
        for (int i = 0; i < r; ++i) fc += (int64_t)legs[i].dir * legs[i].charge(t[i], c);
        ok = vanishes(fc, legs[0].modulus(c));
      }
      if (!ok) continue;
      int64_t b = (int64_t)offset.size();
      int64_t n = 1;
      for (int i = 0; i < r; ++i) {
        qn.push_back(t[i]);
        shape.push_back(legs[i].g[t[i]]);
        n *= legs[i].g[t[i]];
      }
      offset.push_back(off);
      lookup[key_of(t.data(), r)] = b;
      off += n;
      continue;
    }
    flux[depth + 1] = f;
    depth++;
    t[depth] = -1;
  }
  nblocks = (int64_t)offset.size();
  numel = off;
}

int64_t TensorDesc::find(const int32_t* t) const {
  auto it = lookup.find(key_of(t, rank()));
  return it == lookup.end() ? -1 : it->second;
}

int TensorDesc::label_index(const std::string& l) const {
  for (int i = 0; i < rank(); ++i)
    if (legs[i].label == l) return i;
  return -1;
}

std::unique_ptr<TensorDesc> make_tensor(std::vector<LegDesc> legs) {
  if (legs.size() > (size_t)kMaxRank) fail(BST_E_INVALID, "rank above 8");
  for (size_t i = 0; i < legs.size(); ++i) {
    const auto& L = legs[i];
    if (L.dir != 1 && L.dir != -1) fail(BST_E_INVALID, "direction must be +1 or -1");
    if (L.q.empty() || L.q.size() != L.g.size()) fail(BST_E_INVALID, "a leg needs >= 1 sector");
    if (L.sym != legs[0].sym) fail(BST_E_INVALID, "every leg must carry the same symmetries");
    if (L.sym.size() > 8) fail(BST_E_INVALID, "at most 8 symmetries");
    if (L.qx.size() != L.q.size() * (size_t)(L.nsym() - 1))
      fail(BST_E_INVALID, "one charge per symmetry and sector");
    for (int c = 0; c < L.nsym(); ++c) {
      const int32_t n = L.modulus(c);
      if (n < 0 || n == 1) fail(BST_E_INVALID, "a symmetry is U(1) (0) or Z_n with n >= 2");
      if (n >= 2)
        for (size_t k = 0; k < L.q.size(); ++k)
          if (L.charge((int)k, c) < 0 || L.charge((int)k, c) >= n)
            fail(BST_E_QNUM, "a Z_n charge must lie in [0, n)");
    }
    for (auto g : L.g)
      if (g < 1 || g > (int64_t)1 << 30) fail(BST_E_INVALID, "sector dim must be in [1, 2^30]");
    if (L.label.empty()) fail(BST_E_LABEL, "empty label");
    for (size_t j = 0; j < i; ++j)
      if (legs[j].label == L.label) fail(BST_E_LABEL, "duplicate label '" + L.label + "'");
  }
  auto t = std::make_unique<TensorDesc>();
  t->legs = std::move(legs);
  t->build();
  return t;
}

}  // namespace bst

using namespace bst;

namespace bst {
const TensorDesc* desc_of(const bst_tensor* t) { return t ? t->d.get() : nullptr; }
bst_tensor* wrap_tensor(std::unique_ptr<TensorDesc> d) {
  auto* t = new bst_tensor;
  t->d = std::move(d);
  return t;
}
void set_last_error(const std::string& s) { g_last_error = s; }
}  // namespace bst

extern "C" {

const char* bst_last_error(void) { return g_last_error.c_str(); }

const char* bst_version(void) { return "bst 0.1 (gfx950)"; }

bst_status bst_tensor_create(int32_t rank, const int32_t* dir, const int32_t* nsec,
                             const int32_t* qn, const int64_t* dim, const char* const* labels,
                             bst_tensor** out) {
  BST_TRY
  if (!out) fail(BST_E_INVALID, "null output");
  *out = nullptr;
  if (rank < 0 || rank > kMaxRank) fail(BST_E_INVALID, "rank must be 0..8");
  if (rank > 0 && (!dir || !nsec || !qn || !dim || !labels)) fail(BST_E_INVALID, "null argument");
  std::vector<LegDesc> legs(rank);
  int64_t k = 0;
  for (int i = 0; i < rank; ++i) {
    if (nsec[i] < 1) fail(BST_E_INVALID, "a leg needs >= 1 sector");
    legs[i].dir = dir[i];
    if (!labels[i]) fail(BST_E_LABEL, "null label");
    legs[i].label = labels[i];
    for (int s = 0; s < nsec[i]; ++s, ++k) {
      legs[i].q.push_back(qn[k]);
      legs[i].g.push_back(dim[k]);
    }
  }
  *out = wrap_tensor(make_tensor(std::move(legs)));
  BST_CATCH
}

bst_status bst_tensor_create_sym(int32_t rank, const int32_t* dir, const int32_t* nsec, int32_t nsym,
                                 const int32_t* sym, const int32_t* qn, const int64_t* dim,
                                 const char* const* labels, bst_tensor** out) {
  BST_TRY
  if (!out) fail(BST_E_INVALID, "null output");
  *out = nullptr;
  if (rank < 0 || rank > kMaxRank) fail(BST_E_INVALID, "rank must be 0..8");
  if (nsym < 1 || nsym > 8) fail(BST_E_INVALID, "nsym must be 1..8");
  if (!sym) fail(BST_E_INVALID, "null argument");
  if (rank > 0 && (!dir || !nsec || !qn || !dim || !labels)) fail(BST_E_INVALID, "null argument");
  std::vector<int32_t> moduli(sym, sym + nsym);
  std::vector<LegDesc> legs(rank);
  int64_t k = 0;
  for (int i = 0; i < rank; ++i) {
    if (nsec[i] < 1) fail(BST_E_INVALID, "a leg needs >= 1 sector");
    legs[i].dir = dir[i];
    if (!labels[i]) fail(BST_E_LABEL, "null label");
    legs[i].label = labels[i];
    legs[i].sym = moduli;
    for (int s = 0; s < nsec[i]; ++s, ++k) {
      legs[i].q.push_back(qn[k * nsym]);
      for (int c = 1; c < nsym; ++c) legs[i].qx.push_back(qn[k * nsym + c]);
      legs[i].g.push_back(dim[k]);
    }
  }
  *out = wrap_tensor(make_tensor(std::move(legs)));
  BST_CATCH
}

bst_status bst_tensor_symmetry(const bst_tensor* t, int32_t* nsym, int32_t* moduli, int32_t cap) {
  BST_TRY
  if (!t) fail(BST_E_INVALID, "null tensor");
  const int n = t->d->rank() > 0 ? t->d->legs[0].nsym() : 1;
  if (nsym) *nsym = n;
  if (moduli) {
    if (cap < n) fail(BST_E_INVALID, "moduli buffer too small");
    for (int c = 0; c < n; ++c) moduli[c] = t->d->rank() > 0 ? t->d->legs[0].modulus(c) : 0;
  }
  BST_CATCH
}

bst_status bst_tensor_leg_charges(const bst_tensor* t, int32_t leg, int32_t* qn) {
  BST_TRY
  if (!t) fail(BST_E_INVALID, "null tensor");
  if (leg < 0 || leg >= t->d->rank()) fail(BST_E_INVALID, "leg index out of range");
  if (!qn) fail(BST_E_INVALID, "null argument");
  const auto& L = t->d->legs[leg];
  const int n = L.nsym();
  for (size_t s = 0; s < L.q.size(); ++s)
    for (int c = 0; c < n; ++c) qn[s * n + c] = L.charge((int)s, c);
  BST_CATCH
}

bst_status bst_tensor_destroy(bst_tensor* t) {
  delete t;
  g_last_error.clear();
  return BST_OK;
}

bst_status bst_tensor_info(const bst_tensor* t, int32_t* rank, int64_t* nblocks, int64_t* numel) {
  BST_TRY
  if (!t) fail(BST_E_INVALID, "null tensor");
  if (rank) *rank = t->d->rank();
  if (nblocks) *nblocks = t->d->nblocks;
  if (numel) *numel = t->d->numel;
  BST_CATCH
}

bst_status bst_tensor_leg(const bst_tensor* t, int32_t leg, int32_t* dir, int32_t* nsec,
                          int32_t* qn, int64_t* dim, char* label, size_t label_cap) {
  BST_TRY
  if (!t) fail(BST_E_INVALID, "null tensor");
  if (leg < 0 || leg >= t->d->rank()) fail(BST_E_INVALID, "leg index out of range");
  const auto& L = t->d->legs[leg];
  if (dir) *dir = L.dir;
  if (nsec) *nsec = (int32_t)L.q.size();
  if (qn) std::copy(L.q.begin(), L.q.end(), qn);
  if (dim) std::copy(L.g.begin(), L.g.end(), dim);
  if (label) {
    if (label_cap < L.label.size() + 1) fail(BST_E_INVALID, "label buffer too small");
    std::memcpy(label, L.label.c_str(), L.label.size() + 1);
  }
  BST_CATCH
}

bst_status bst_tensor_block(const bst_tensor* t, int64_t b, int32_t* qn_idx, int64_t* shape,
                            int64_t* offset) {
  BST_TRY
  if (!t) fail(BST_E_INVALID, "null tensor");
  const auto& d = *t->d;
  if (b < 0 || b >= d.nblocks) fail(BST_E_INVALID, "block index out of range");
  int r = d.rank();
  if (qn_idx) std::copy(d.block_qn(b), d.block_qn(b) + r, qn_idx);
  if (shape) std::copy(d.block_shape(b), d.block_shape(b) + r, shape);
  if (offset) *offset = d.offset[b];
  BST_CATCH
}

bst_status bst_tensor_find_block(const bst_tensor* t, const int32_t* qn_idx, int64_t* b) {
  BST_TRY
  if (!t || !b) fail(BST_E_INVALID, "null argument");
  const auto& d = *t->d;
  if (d.rank() > 0 && !qn_idx) fail(BST_E_INVALID, "null qn_idx");
  for (int i = 0; i < d.rank(); ++i)
    if (qn_idx[i] < 0 || qn_idx[i] >= (int32_t)d.legs[i].q.size())
      fail(BST_E_INVALID, "Qn index out of range");
  int64_t r = d.find(qn_idx);
  if (r < 0) fail(BST_E_NOBLOCK, "no valid block with these Qn indices (nonzero flux)");
  *b = r;
  BST_CATCH
}

}  // extern "C"

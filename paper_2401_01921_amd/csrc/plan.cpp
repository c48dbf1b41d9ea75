// Plan builders: charge-sector matching for permute, pairwise contraction
// and the two-site H_eff, all exact integer work done once per structure.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <numeric>

namespace bst {

static std::atomic<uint64_t> g_plan_id{1};

static void check_contractible(const LegDesc& a, const LegDesc& b, const std::string& what) {
  if (a.dir == b.dir)
    fail(BST_E_DIRECTION, "leg '" + what + "' has the same direction on both tensors");
  if (a.sym != b.sym) fail(BST_E_QNUM, "leg '" + what + "' has different symmetries");
  if (!a.same_charges(b)) fail(BST_E_QNUM, "leg '" + what + "' has different quantum numbers");
  if (a.g != b.g) fail(BST_E_DIM, "leg '" + what + "' has different sector dims");
}

static void check_same(const LegDesc& a, const LegDesc& b, const std::string& what) {
  if (a.dir != b.dir || !a.same_sectors(b))
    fail(BST_E_STRUCTURE, "leg '" + what + "' of the result does not match psi");
}

// ------------------------------------------------------------------------
// Permute jobs
// ------------------------------------------------------------------------
// Appends the jobs that move every block of `in` (slot in_slot) to its place
// in `out` = in with legs permuted by perm (new leg i = old leg perm[i]).
static void add_permute_jobs(Step& st, const TensorDesc& in, const TensorDesc& out,
                             const std::vector<int>& perm, int in_slot, int out_slot) {
  const int r = in.rank();
  std::vector<int> pos(r);
  for (int k = 0; k < r; ++k) pos[perm[k]] = k;
  std::vector<int32_t> nt(r);
  for (int64_t b = 0; b < in.nblocks; ++b) {
    const int32_t* t = in.block_qn(b);
    for (int k = 0; k < r; ++k) nt[k] = t[perm[k]];
    const int64_t ob = out.find(nt.data());
    if (ob < 0) fail(BST_E_INVALID, "internal: permuted block missing");
    const int64_t* sh = in.block_shape(b);
    // output strides of the output block (row-major over the permuted shape)
    std::vector<int64_t> ostr_out(r, 1);
    for (int k = r - 2; k >= 0; --k) ostr_out[k] = ostr_out[k + 1] * sh[perm[k + 1]];
    // reduce: drop size-1 dims, merge input-adjacent dims that stay adjacent
    std::vector<int64_t> ext;
    std::vector<int64_t> ost;
    std::vector<int> opos;
    for (int d = 0; d < r; ++d) {
      if (sh[d] == 1) continue;
      if (!ext.empty() && opos.back() + 1 == pos[d]) {
        // check that no non-unit output dim sits between them (pos adjacent ensures it)
        ext.back() *= sh[d];
        ost.back() = ostr_out[pos[d]];
        opos.back() = pos[d];
        continue;
      }
      ext.push_back(sh[d]);
      ost.push_back(ostr_out[pos[d]]);
      opos.push_back(pos[d]);
    }
    if (ext.empty()) {
      ext.push_back(1);
      ost.push_back(1);
    }
    const int rr = (int)ext.size();
    PermJob j{};
    j.in_off = in.offset[b];
    j.out_off = out.offset[ob];
    j.in_buf = in_slot;
    j.out_buf = out_slot;
    j.rank = rr;
    int64_t s = 1;
    for (int d = rr - 1; d >= 0; --d) {
      j.shape[d] = (int32_t)ext[d];
      j.istride[d] = s;
      j.ostride[d] = ost[d];
      s *= ext[d];
    }
    j.pdim = -1;
    for (int d = 0; d < rr; ++d)
      if (ost[d] == 1 && ext[d] > 1) j.pdim = d;
    const int jid = (int)st.jobs.size();
    const int64_t last = ext[rr - 1];
    const int64_t numel = s;
    if (rr == 1 || j.pdim == rr - 1 || j.pdim < 0) {
      j.pdim = rr - 1;
      st.jobs.push_back(j);
      const int64_t rows = numel / last;
      int64_t per = std::max<int64_t>(1, 8192 / last);
      per = std::min<int64_t>(per, kPermRows);
      for (int64_t r0 = 0; r0 < rows; r0 += per) {
        PermWork w{};
        w.job = jid;
        w.kind = 0;
        w.batch = r0;
        w.t0 = (int32_t)std::min<int64_t>(per, rows - r0);
        st.pwork.push_back(w);
      }
    } else {
      st.jobs.push_back(j);
      const int64_t np = ext[j.pdim];
      int64_t nbatch = numel / (np * last);
      // 64 x 64 tiles; a last strip of the last dim no wider than 32 (16)
      // elements goes in 128 x 32 (256 x 16) tiles, so that few lanes idle
      // (strip by strip of the last dim: measured 4.30 TB/s against 4.19
      // with the tiles of one row band consecutive)
      for (int64_t bt = 0; bt < nbatch; ++bt)
        for (int64_t x = 0; x < last; x += 64) {
          const int64_t wx = std::min<int64_t>(64, last - x);
          const int kind = wx > 32 ? 1 : wx > 16 ? 2 : 3;
          const int64_t ty = kind == 1 ? 64 : kind == 2 ? 128 : 256;
          for (int64_t y = 0; y < np; y += ty) {
            PermWork w{};
            w.job = jid;
            w.kind = kind;
            w.batch = bt;
            w.t0 = (int32_t)y;
            w.t1 = (int32_t)x;
            st.pwork.push_back(w);
          }
        }
    }
  }
  st.bytes += 16.0 * (double)in.numel;
  st.bytes32 += 16.0 * (double)in.numel;
}

static std::unique_ptr<TensorDesc> permuted_desc(const TensorDesc& in, const std::vector<int>& perm) {
  std::vector<LegDesc> legs;
  for (int k : perm) legs.push_back(in.legs[k]);
  return make_tensor(std::move(legs));
}

// ------------------------------------------------------------------------
// Pairwise contraction (Sec. "Tensor contraction")
// ------------------------------------------------------------------------
struct ContractBuild {
  std::unique_ptr<TensorDesc> C;
  std::unique_ptr<TensorDesc> Apack, Bpack;   // null if the operand is used in place
  std::vector<int> permA, permB;
};

// Fills `st` (a GEMM step) for C = A . B with A given as [free.., contracted..]
// (tensor Ause, slot a_slot) and B as [contracted.., free..] (NN) or
// [free.., contracted..] (NT).
static void build_gemm(Step& st, const TensorDesc& Ause, int a_slot, int na_free,
                       const TensorDesc& Buse, int b_slot, int nb_free, bool transb,
                       const TensorDesc& C, int c_slot) {
  const int ra = Ause.rank(), rb = Buse.rank();
  const int nc = ra - na_free;
  // index A blocks by free tuple
  std::unordered_map<std::string, std::vector<int64_t>> a_by_free;
  for (int64_t b = 0; b < Ause.nblocks; ++b) {
    const int32_t* t = Ause.block_qn(b);
    a_by_free[std::string(reinterpret_cast<const char*>(t), 4 * na_free)].push_back(b);
  }
  std::vector<int32_t> bt(rb);
  st.kind = StepKind::Gemm;
  st.transb = transb;
  for (int64_t cb = 0; cb < C.nblocks; ++cb) {
    const int32_t* ct = C.block_qn(cb);
    const int64_t* cs = C.block_shape(cb);
    GemmProb p{};
    int64_t M = 1, N = 1;
    for (int i = 0; i < na_free; ++i) M *= cs[i];
    for (int i = 0; i < nb_free; ++i) N *= cs[na_free + i];
    if (M > 0x7FFFFFFF || N > 0x7FFFFFFF) fail(BST_E_INVALID, "block too large");
    p.c_off = C.offset[cb];
    p.c_buf = c_slot;
    p.M = (int32_t)M;
    p.N = (int32_t)N;
    p.ldc = (int32_t)N;
    p.seg_begin = (int32_t)st.segs.size();
    auto it = a_by_free.find(std::string(reinterpret_cast<const char*>(ct), 4 * na_free));
    if (it != a_by_free.end()) {
      for (int64_t ab : it->second) {
        const int32_t* at = Ause.block_qn(ab);
        // B tuple
        if (!transb) {
          for (int i = 0; i < nc; ++i) bt[i] = at[na_free + i];
          for (int i = 0; i < nb_free; ++i) bt[nc + i] = ct[na_free + i];
        } else {
          for (int i = 0; i < nb_free; ++i) bt[i] = ct[na_free + i];
          for (int i = 0; i < nc; ++i) bt[nb_free + i] = at[na_free + i];
        }
        const int64_t bb = Buse.find(bt.data());
        if (bb < 0) continue;
        int64_t K = 1;
        for (int i = 0; i < nc; ++i) K *= Ause.block_shape(ab)[na_free + i];
        if (K > 0x7FFFFFFF) fail(BST_E_INVALID, "block too large");
        GemmSeg g{};
        g.a_off = Ause.offset[ab];
        g.a_buf = a_slot;
        g.b_off = Buse.offset[bb];
        g.b_buf = b_slot;
        g.K = (int32_t)K;
        g.lda = (int32_t)K;
        g.ldb = transb ? (int32_t)K : (int32_t)N;
        st.segs.push_back(g);
        st.flops += 2.0 * (double)M * (double)N * (double)K;
      }
    }
    p.seg_count = (int32_t)st.segs.size() - p.seg_begin;
    st.probs.push_back(p);
  }
}

static void contract_plan(const TensorDesc& A, const TensorDesc& B, PlanData& P,
                          std::unique_ptr<TensorDesc>& Cout) {
  const int ra = A.rank(), rb = B.rank();
  std::vector<int> ac, bc;
  for (int i = 0; i < ra; ++i) {
    int j = B.label_index(A.legs[i].label);
    if (j >= 0) {
      check_contractible(A.legs[i], B.legs[j], A.legs[i].label);
      ac.push_back(i);
      bc.push_back(j);
    }
  }
  std::vector<int> af, bf;
  for (int i = 0; i < ra; ++i)
    if (std::find(ac.begin(), ac.end(), i) == ac.end()) af.push_back(i);
  for (int j = 0; j < rb; ++j)
    if (std::find(bc.begin(), bc.end(), j) == bc.end()) bf.push_back(j);
  std::vector<LegDesc> cl;
  for (int i : af) cl.push_back(A.legs[i]);
  for (int j : bf) cl.push_back(B.legs[j]);
  // the output's labels must be unique
  Cout = make_tensor(cl);
  const TensorDesc& C = *Cout;

  P.kind = 1;
  P.in_slots = {0, 1};
  P.out_slots = {2};
  P.in_numel = {A.numel, B.numel};
  P.out_numel = {C.numel};
  P.nslots = 3;
  // A operand: [free.., contracted..]
  std::vector<int> permA = af;
  permA.insert(permA.end(), ac.begin(), ac.end());
  bool packA = false;
  for (int i = 0; i < ra; ++i)
    if (permA[i] != i) packA = true;
  // B operand
  std::vector<int> nn = bc;
  nn.insert(nn.end(), bf.begin(), bf.end());
  std::vector<int> nt = bf;
  nt.insert(nt.end(), bc.begin(), bc.end());
  auto is_identity = [](const std::vector<int>& v) {
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] != (int)i) return false;
    return true;
  };
  bool transb = false, packB = false;
  if (is_identity(nn)) {
    transb = false;
  } else if (is_identity(nt)) {
    transb = true;
  } else {
    packB = true;
  }
  std::unique_ptr<TensorDesc> Ap, Bp;
  int a_slot = 0, b_slot = 1;
  if (packA) {
    Ap = permuted_desc(A, permA);
    Step st;
    st.kind = StepKind::Permute;
    st.name = "pack_a";
    a_slot = P.nslots++;
    P.internals.push_back({a_slot, (size_t)A.numel * 8, 0});
    add_permute_jobs(st, A, *Ap, permA, 0, a_slot);
    P.steps.push_back(std::move(st));
  }
  if (packB) {
    Bp = permuted_desc(B, nn);
    Step st;
    st.kind = StepKind::Permute;
    st.name = "pack_b";
    b_slot = P.nslots++;
    P.internals.push_back({b_slot, (size_t)B.numel * 8, 0});
    add_permute_jobs(st, B, *Bp, nn, 1, b_slot);
    P.steps.push_back(std::move(st));
  }
  Step g;
  g.name = "gemm";
  build_gemm(g, packA ? *Ap : A, a_slot, (int)af.size(), packB ? *Bp : B, b_slot, (int)bf.size(),
             transb, C, 2);
  g.bytes = 8.0 * ((double)A.numel + (double)B.numel + (double)C.numel);
  g.bytes32 = g.bytes;
  P.steps.push_back(std::move(g));
}

// ------------------------------------------------------------------------
// Complex float64 data (Sec. "Creating a non-symmetric UniTensor",
// paragraph "Complex elements and data types"; App. "Quantum Circuit
// Simulation" works on complex tensors).  A complex tensor
// stores each element as two float64, real then imaginary: its flat buffer
// is that of the real tensor with one more, fastest leg of dim 2 (charge 0).
// A permute keeps that leg last.  A contraction A.B is the real contraction
// of A in that interleaved form with B expanded element by element into the
// 2 x 2 block [[Br, Bi], [-Bi, Br]] (legs: B's contracted legs, the re/im leg
// that meets A's, B's free legs, the output's re/im leg), which gives C in
// the interleaved form: sum_k (Ar Br - Ai Bi, Ar Bi + Ai Br).
// ------------------------------------------------------------------------
static const char* const kReLabel = "#re";
static const char* const kReOutLabel = "#re'";

static LegDesc reim_leg(const LegDesc& like, int dir, const char* label) {
  LegDesc l;
  l.dir = dir;
  l.sym = like.sym;
  l.q = {0};
  for (int c = 1; c < like.nsym(); ++c) l.qx.push_back(0);
  l.g = {2};
  l.label = label;
  return l;
}

static void check_complex(const TensorDesc& T, int max_rank) {
  if (T.rank() < 1) fail(BST_E_INVALID, "complex tensors need rank >= 1");
  if (T.rank() > max_rank)
    fail(BST_E_INVALID, "complex tensors of this operation are limited to rank " + std::to_string(max_rank));
  for (const auto& l : T.legs)
    if (l.label.compare(0, 3, "#re") == 0) fail(BST_E_LABEL, "labels starting with '#re' are reserved");
}

static std::unique_ptr<TensorDesc> with_reim(const TensorDesc& T) {
  std::vector<LegDesc> legs = T.legs;
  legs.push_back(reim_leg(T.legs[0], 1, kReLabel));
  return make_tensor(std::move(legs));
}

static void permute_c128_plan(const TensorDesc& T, const std::vector<int>& perm, PlanData& P,
                              std::unique_ptr<TensorDesc>& out) {
  check_complex(T, kMaxRank - 1);
  auto Tr = with_reim(T);
  std::vector<int> pr = perm;
  pr.push_back(T.rank());
  auto Or = permuted_desc(*Tr, pr);
  P.kind = 0;
  P.in_slots = {0};
  P.out_slots = {1};
  P.in_numel = {Tr->numel};
  P.out_numel = {Or->numel};
  P.nslots = 2;
  Step st;
  st.kind = StepKind::Permute;
  st.name = "permute";
  add_permute_jobs(st, *Tr, *Or, pr, 0, 1);
  P.steps.push_back(std::move(st));
  out = permuted_desc(T, perm);
}

static void contract_c128_plan(const TensorDesc& A, const TensorDesc& B, PlanData& P,
                               std::unique_ptr<TensorDesc>& Cout) {
  check_complex(A, kMaxRank - 1);
  check_complex(B, kMaxRank - 2);
  std::vector<int> ac, bc, bf;
  for (int i = 0; i < A.rank(); ++i) {
    const int j = B.label_index(A.legs[i].label);
    if (j < 0) continue;
    check_contractible(A.legs[i], B.legs[j], A.legs[i].label);
    ac.push_back(i);
    bc.push_back(j);
  }
  for (int j = 0; j < B.rank(); ++j)
    if (std::find(bc.begin(), bc.end(), j) == bc.end()) bf.push_back(j);
  const int nc = (int)bc.size();
  if (A.rank() + B.rank() - 2 * nc + 1 > kMaxRank)
    fail(BST_E_INVALID, "complex contraction output limited to rank " + std::to_string(kMaxRank - 1));
  // B in [contracted (A's order).., free..] order, then expanded
  std::vector<int> permB = bc;
  permB.insert(permB.end(), bf.begin(), bf.end());
  auto Bp = permuted_desc(B, permB);
  std::vector<LegDesc> xl(Bp->legs.begin(), Bp->legs.begin() + nc);
  xl.push_back(reim_leg(B.legs[0], -1, kReLabel));
  xl.insert(xl.end(), Bp->legs.begin() + nc, Bp->legs.end());
  xl.push_back(reim_leg(B.legs[0], -1, kReOutLabel));
  auto Bx = make_tensor(std::move(xl));
  auto Ar = with_reim(A);
  std::unique_ptr<TensorDesc> Cr;
  contract_plan(*Ar, *Bx, P, Cr);   // slots: 0 A (interleaved), 1 B', 2 C (interleaved)
  for (const auto& st : P.steps)
    if (st.name == "pack_b") fail(BST_E_INVALID, "internal: expanded B is not in GEMM order");
  std::vector<Step> pre;
  int src = 1;
  bool ident = true;
  for (int i = 0; i < (int)permB.size(); ++i) ident = ident && permB[i] == i;
  if (!ident) {
    auto Br = with_reim(B);
    std::vector<int> pr = permB;
    pr.push_back(B.rank());
    auto Bpr = permuted_desc(*Br, pr);
    Step st;
    st.kind = StepKind::Permute;
    st.name = "pack_b";
    src = P.nslots++;
    P.internals.push_back({src, (size_t)Bpr->numel * 8, 0});
    add_permute_jobs(st, *Br, *Bpr, pr, 1, src);
    pre.push_back(std::move(st));
  }
  Step ex;
  ex.kind = StepKind::Expand;
  ex.name = "expand_b";
  const int xslot = P.nslots++;
  P.internals.push_back({xslot, (size_t)Bx->numel * 8, 0});
  std::vector<int32_t> xt(Bx->rank());
  for (int64_t b = 0; b < Bp->nblocks; ++b) {
    const int32_t* t = Bp->block_qn(b);
    const int64_t* sh = Bp->block_shape(b);
    int64_t K = 1, N = 1;
    for (int i = 0; i < nc; ++i) K *= sh[i];
    for (int i = nc; i < Bp->rank(); ++i) N *= sh[i];
    if (K > 0x7FFFFFFF || N > 0x7FFFFFFF) fail(BST_E_INVALID, "block too large");
    for (int i = 0; i < nc; ++i) xt[i] = t[i];
    xt[nc] = 0;
    for (int i = nc; i < Bp->rank(); ++i) xt[i + 1] = t[i];
    xt[Bx->rank() - 1] = 0;
    const int64_t xb = Bx->find(xt.data());
    if (xb < 0) fail(BST_E_INVALID, "internal: expanded block missing");
    const int32_t jid = (int32_t)ex.xjobs.size();
    ex.xjobs.push_back({2 * Bp->offset[b], Bx->offset[xb], src, xslot, (int32_t)K, (int32_t)N});
    for (int64_t st0 = 0; st0 < K * N; st0 += 4096) ex.xwork.push_back({jid, (int32_t)st0});
  }
  ex.bytes = ex.bytes32 = 16.0 * (double)Bp->numel + 32.0 * (double)Bp->numel;
  pre.push_back(std::move(ex));
  // the contraction now reads B' from its internal slot
  for (auto& st : P.steps)
    for (auto& g : st.segs)
      if (g.b_buf == 1) g.b_buf = xslot;
  P.steps.insert(P.steps.begin(), std::make_move_iterator(pre.begin()), std::make_move_iterator(pre.end()));
  P.in_numel = {Ar->numel, 2 * B.numel};
  std::vector<LegDesc> cl(Cr->legs.begin(), Cr->legs.end() - 1);
  Cout = make_tensor(std::move(cl));
}

// ------------------------------------------------------------------------
// Two-site H_eff (Sec. "Benchmarks", Fig. Hpsi_fig)
// ------------------------------------------------------------------------
// Dense index -> (sector, index in sector) of a leg.
struct LegMap {
  std::vector<int32_t> sec, within;
  std::vector<int64_t> start;
  explicit LegMap(const LegDesc& L) {
    int64_t s = 0;
    for (size_t k = 0; k < L.g.size(); ++k) {
      start.push_back(s);
      for (int64_t e = 0; e < L.g[k]; ++e) {
        sec.push_back((int32_t)k);
        within.push_back((int32_t)e);
      }
      s += L.g[k];
    }
  }
};

// Flat offset of a dense element of a rank-4 tensor, -1 outside valid blocks.
static int64_t elem_offset4(const TensorDesc& T, const LegMap* maps, const int64_t* idx) {
  int32_t t[4];
  for (int i = 0; i < 4; ++i) t[i] = maps[i].sec[idx[i]];
  const int64_t b = T.find(t);
  if (b < 0) return -1;
  const int64_t* sh = T.block_shape(b);
  int64_t off = 0;
  for (int i = 0; i < 4; ++i) off = off * sh[i] + maps[i].within[idx[i]];
  return T.offset[b] + off;
}

// bfloat16-plane layout of a tensor seen as a matrix per block: rows are the
// first `split` legs, columns the rest; rows (or, transposed, columns) are
// padded to a multiple of 32 elements (one 32-deep k step), so every row of
// every block starts on a 32-element bound.  Positions are planar; the
// planes are interleaved by chunks (plane_at).
struct PadLayout {
  std::vector<int64_t> off, ld;
  int64_t total = 0;   // positions per plane, a multiple of 32
};
static int64_t pad8(int64_t x) { return (x + 7) / 8 * 8; }
static int64_t pad32(int64_t x) { return (x + 31) / 32 * 32; }

static void block_matrix(const TensorDesc& T, int64_t b, int split, int64_t& rows, int64_t& cols) {
  rows = 1;
  cols = 1;
  for (int i = 0; i < T.rank(); ++i) (i < split ? rows : cols) *= T.block_shape(b)[i];
}

static PadLayout pad_layout(const TensorDesc& T, int split, bool transpose) {
  PadLayout P;
  int64_t cum = 0;
  for (int64_t b = 0; b < T.nblocks; ++b) {
    int64_t rows, cols;
    block_matrix(T, b, split, rows, cols);
    const int64_t ld = transpose ? pad32(rows) : pad32(cols);
    P.off.push_back(cum);
    P.ld.push_back(ld);
    cum += (transpose ? cols : rows) * ld;
  }
  P.total = pad32(std::max<int64_t>(cum, 32));
  return P;
}

// Like pad_layout (not transposed), with the blocks ordered by their sector
// on leg `group_leg` (canonical order inside a group), so that the blocks
// sharing that sector form one matrix of stacked rows.  gstart[k] is the
// offset of group k, grow[b] the first row of block b inside its group and
// gm[k] the rows of group k.
struct GroupedLayout {
  PadLayout lay;
  std::vector<int64_t> gstart, gm, grow;
};

static GroupedLayout pad_layout_grouped(const TensorDesc& T, int split, int group_leg) {
  GroupedLayout G;
  const int ng = (int)T.legs[group_leg].q.size();
  G.lay.off.assign(T.nblocks, 0);
  G.lay.ld.assign(T.nblocks, 0);
  G.grow.assign(T.nblocks, 0);
  G.gstart.assign(ng, 0);
  G.gm.assign(ng, 0);
  int64_t cum = 0;
  for (int k = 0; k < ng; ++k) {
    G.gstart[k] = cum;
    for (int64_t b = 0; b < T.nblocks; ++b) {
      if (T.block_qn(b)[group_leg] != k) continue;
      int64_t rows, cols;
      block_matrix(T, b, split, rows, cols);
      const int64_t ld = pad32(cols);
      G.lay.off[b] = cum;
      G.lay.ld[b] = ld;
      G.grow[b] = G.gm[k];
      G.gm[k] += rows;
      cum += rows * ld;
    }
  }
  G.lay.total = pad32(std::max<int64_t>(cum, 32));
  return G;
}

static void add_split_jobs(Step& st, const TensorDesc& T, int split, bool transpose,
                           const PadLayout& Lay, int in_slot, int out_slot) {
  st.kind = StepKind::Split;
  for (int64_t b = 0; b < T.nblocks; ++b) {
    int64_t rows, cols;
    block_matrix(T, b, split, rows, cols);
    if (rows > 0x7FFFFFFF || cols > 0x7FFFFFFF || Lay.ld[b] > 0x7FFFFFFF)
      fail(BST_E_INVALID, "block too large for the bfloat16 split");
    SplitJob j{};
    j.in_off = T.offset[b];
    j.out_off = Lay.off[b];
    j.in_buf = in_slot;
    j.out_buf = out_slot;
    j.rows = (int32_t)rows;
    j.cols = (int32_t)cols;
    j.out_ld = (int32_t)Lay.ld[b];
    j.transpose = transpose ? 1 : 0;
    const int32_t jid = (int32_t)st.sjobs.size();
    st.sjobs.push_back(j);
    const int64_t rext = transpose ? Lay.ld[b] : rows;
    const int64_t cext = transpose ? cols : Lay.ld[b];
    for (int64_t r0 = 0; r0 < rext; r0 += 64)
      for (int64_t c0 = 0; c0 < cext; c0 += 64) st.swork.push_back({jid, (int32_t)r0, (int32_t)c0, 0});
  }
  st.bytes += 8.0 * (double)T.numel + 4.0 * (double)Lay.total;
  st.bytes32 = st.bytes;
}

static void heff_plan(const TensorDesc& L, const TensorDesc& W1, const TensorDesc& W2,
                      const TensorDesc& R, const TensorDesc& psi, PlanData& P) {
  if (L.rank() != 3 || W1.rank() != 4 || W2.rank() != 4 || R.rank() != 3 || psi.rank() != 4)
    fail(BST_E_STRUCTURE, "H_eff needs L[a,w,a'], W[wl,s,s',wr] (x2), R[b,w,b'], psi[a,s1,s2,b]");
  check_contractible(L.legs[2], psi.legs[0], "L.a' / psi.a");
  check_contractible(L.legs[1], W1.legs[0], "L.w / W1.wl");
  check_contractible(W1.legs[2], psi.legs[1], "W1.s' / psi.s1");
  check_contractible(W1.legs[3], W2.legs[0], "W1.wr / W2.wl");
  check_contractible(W2.legs[2], psi.legs[2], "W2.s' / psi.s2");
  check_contractible(W2.legs[3], R.legs[1], "W2.wr / R.w");
  check_contractible(R.legs[2], psi.legs[3], "R.b' / psi.b");
  check_same(L.legs[0], psi.legs[0], "a");
  check_same(W1.legs[1], psi.legs[1], "s1");
  check_same(W2.legs[1], psi.legs[2], "s2");
  check_same(R.legs[0], psi.legs[3], "b");

  // slots: 0 L, 1 W1, 2 W2, 3 R, 4 psi, 5 out, 6 T1, 7 T3
  P.kind = 2;
  P.in_slots = {0, 1, 2, 3, 4};
  P.out_slots = {5};
  P.in_numel = {L.numel, W1.numel, W2.numel, R.numel, psi.numel};
  P.out_numel = {psi.numel};
  P.nslots = 8;
  P.psi_numel = psi.numel;

  auto lab = [](LegDesc l, const char* s) {
    l.label = s;
    return l;
  };
  // T1[a, w1, t1, t2, y] and T3[a, s1, s2, w3, y]
  auto T1 = make_tensor({lab(L.legs[0], "a"), lab(L.legs[1], "w1"), lab(psi.legs[1], "t1"),
                         lab(psi.legs[2], "t2"), lab(psi.legs[3], "y")});
  auto T3 = make_tensor({lab(psi.legs[0], "a"), lab(W1.legs[1], "s1"), lab(W2.legs[1], "s2"),
                         lab(W2.legs[3], "w3"), lab(psi.legs[3], "y")});
  P.t1_numel = T1->numel;
  P.t3_numel = T3->numel;
  P.internals.push_back({6, (size_t)T1->numel * 8, 0});
  P.internals.push_back({7, (size_t)T3->numel * 8, 0});
  // bfloat16 planes for the split forms: L [(a w) x a'], R [b x (w b')],
  // psi transposed to [(t1 t2 b') x a'], T3 [(a s1 s2) x (w3 b')]
  P.has_planes = true;
  P.nslots = 12;
  // L's planes are grouped by the contracted sector a' so that all L rows
  // meeting one psi sector a' form one matrix (step 1 then runs one GEMM per
  // a' sector); psi's transposed blocks are already grouped by a'.
  const GroupedLayout Lg = pad_layout_grouped(L, 2, 2);
  const PadLayout& Lp = Lg.lay;
  const PadLayout Rp = pad_layout(R, 1, false), Pp = pad_layout(psi, 1, true);
  // T3 planes in a merged layout for step 4: per output sector b, one matrix
  // whose rows are all psi blocks (a, s1, s2, b) stacked and whose columns
  // are the K-segments (w3, b') of R's blocks (b, w3, b'), each segment
  // starting at a multiple of 8 elements.
  const int nB = (int)psi.legs[3].q.size();
  std::vector<int64_t> t3g(nB, 0), t3w(nB, 0), t3m(nB, 0), prow(psi.nblocks, 0),
      rseg(R.nblocks, 0);
  int64_t t3tot = 0;
  for (int kb = 0; kb < nB; ++kb) {
    for (int64_t b = 0; b < psi.nblocks; ++b) {
      if (psi.block_qn(b)[3] != kb) continue;
      prow[b] = t3m[kb];
      t3m[kb] += psi.block_shape(b)[0] * psi.block_shape(b)[1] * psi.block_shape(b)[2];
    }
    for (int64_t b = 0; b < R.nblocks; ++b) {
      if (R.block_qn(b)[0] != kb) continue;
      rseg[b] = t3w[kb];
      t3w[kb] += pad32(R.block_shape(b)[1] * R.block_shape(b)[2]);
    }
    t3g[kb] = t3tot;
    t3tot += t3m[kb] * t3w[kb];
  }
  // T3 blocks that no output sector b reads (w3 + b' charge outside b's
  // sectors) are still produced by the MPO step; their planes all go to
  // one write-only sink after the groups, which step 4 never reads.
  const int64_t t3sink = t3tot;
  int64_t sink_need = 0;
  for (int64_t b = 0; b < T3->nblocks; ++b) {
    const int64_t* sh = T3->block_shape(b);
    sink_need = std::max(sink_need, sh[0] * sh[4]);
  }
  const int64_t t3ps = pad32(std::max<int64_t>(t3tot + sink_need, 32));   // positions per plane
  // 8 bytes per position: three bfloat16 planes or one of float64
  P.internals.push_back({8, (size_t)Lp.total * 8, 0});
  P.internals.push_back({9, (size_t)Rp.total * 8, 0});
  P.internals.push_back({10, (size_t)Pp.total * 8, 0});
  P.internals.push_back({11, (size_t)t3ps * 8, 0});
  Step spL, spR, spP;
  spL.name = "split_L";
  spR.name = "split_R";
  spP.name = "split_psi";
  add_split_jobs(spL, L, 2, false, Lp, 0, 8);
  add_split_jobs(spR, R, 1, false, Rp, 3, 9);
  add_split_jobs(spP, psi, 1, true, Pp, 4, 10);
  spP.reads_psi = true;
  spL.constant = spR.constant = true;

  // merged T1 layout of the plane variant (filled with step 1)
  std::vector<int64_t> t1m_start, t1m_ld, pcol, t1zero;

  // ---- step 1: T1[(a w) x (t1 t2 y)] = sum_a' L[(a w) x a'] psi[a' x (t1 t2 y)]
  Step s1;
  s1.kind = StepKind::Gemm;
  s1.name = "gemm_L_psi";
  s1.tc = Elem::Inter;
  s1.has_alt = true;
  s1.fusable = true;
  {
    const int nA = (int)psi.legs[0].q.size();
    int32_t lt[3], pt[4];
    for (int64_t cb = 0; cb < T1->nblocks; ++cb) {
      const int32_t* t = T1->block_qn(cb);
      const int64_t* sh = T1->block_shape(cb);
      GemmProb p{};
      const int64_t M = sh[0] * sh[1], N = sh[2] * sh[3] * sh[4];
      p.c_off = T1->offset[cb];
      p.c_buf = 6;
      p.M = (int32_t)M;
      p.N = (int32_t)N;
      p.ldc = (int32_t)N;
      p.seg_begin = (int32_t)s1.segs.size();
      for (int kap = 0; kap < nA; ++kap) {
        lt[0] = t[0]; lt[1] = t[1]; lt[2] = kap;
        pt[0] = kap; pt[1] = t[2]; pt[2] = t[3]; pt[3] = t[4];
        const int64_t lb = L.find(lt), pb = psi.find(pt);
        if (lb < 0 || pb < 0) continue;
        GemmSeg g{};
        const int64_t K = psi.legs[0].g[kap];
        g.a_off = L.offset[lb];
        g.a_buf = 0;
        g.b_off = psi.offset[pb];
        g.b_buf = 4;
        g.K = (int32_t)K;
        g.lda = (int32_t)K;
        g.ldb = (int32_t)N;
        s1.segs.push_back(g);
        s1.flops += 2.0 * (double)M * (double)N * (double)K;
      }
      p.seg_count = (int32_t)s1.segs.size() - p.seg_begin;
      s1.probs.push_back(p);
    }
    s1.segs_alt.clear();
    // plane variant: one problem per a' sector kx.  Rows: every L block
    // (a, w, kx) stacked (grouped L planes); columns: every psi block
    // (kx, t1, t2, y) stacked (transposed psi planes); the result is T1 in a
    // merged layout, [rows x columns] per kx, read back by the MPO step;
    // rows padded to 16 floats, so that the GEMM's 64-byte row stores are
    // whole 64-byte blocks.
    t1m_start.assign(nA, 0);
    t1m_ld.assign(nA, 0);
    pcol.assign(psi.nblocks, 0);
    int64_t cum = 0;
    for (int kx = 0; kx < nA; ++kx) {
      int64_t ncol = 0, pfirst = -1;
      for (int64_t b = 0; b < psi.nblocks; ++b) {
        if (psi.block_qn(b)[0] != kx) continue;
        if (pfirst < 0) pfirst = b;
        pcol[b] = ncol;
        int64_t rows, cols;
        block_matrix(psi, b, 1, rows, cols);
        ncol += cols;
      }
      t1m_start[kx] = cum;
      t1m_ld[kx] = (ncol + 15) / 16 * 16;
      const int64_t M = Lg.gm[kx];
      cum += M * t1m_ld[kx];
      if (M == 0 || ncol == 0) continue;
      if (M > 0x7FFFFFFF || ncol > 0x7FFFFFFF) fail(BST_E_INVALID, "sector group too large");
      const int64_t K = psi.legs[0].g[kx];
      GemmProb p{};
      p.c_off = t1m_start[kx];
      p.c_buf = 6;
      p.M = (int32_t)M;
      p.N = (int32_t)ncol;
      p.ldc = (int32_t)t1m_ld[kx];
      p.seg_begin = (int32_t)s1.segs_alt.size();
      p.seg_count = 1;
      GemmSeg h{};
      h.a_off = Lg.gstart[kx];
      h.a_buf = 8;
      h.lda = (int32_t)pad32(K);
      h.b_off = Pp.off[pfirst];
      h.b_buf = 10;
      h.ldb = (int32_t)pad32(K);
      h.K = (int32_t)K;
      s1.segs_alt.push_back(h);
      s1.probs_alt.push_back(p);
    }
    // T1 blocks that no (L, psi) pair reaches stay zero: each gets a region
    // of its own, written (as zeros) by a problem without segments
    t1zero.assign(T1->nblocks, -1);
    for (int64_t cb = 0; cb < T1->nblocks; ++cb) {
      if (s1.probs[cb].seg_count > 0) continue;
      t1zero[cb] = cum;
      GemmProb p = s1.probs[cb];
      p.c_off = cum;
      p.seg_begin = (int32_t)s1.segs_alt.size();
      p.seg_count = 0;
      s1.probs_alt.push_back(p);
      cum += T1->block_size(cb);
    }
    // the T1 buffer holds the float64 block layout or this merged one (float32
    // for the split forms, float64 for the float64 panels)
    for (auto& ib : P.internals)
      if (ib.slot == 6) ib.bytes = std::max(ib.bytes, (size_t)cum * 8);
    s1.bytes = 8.0 * ((double)L.numel + (double)psi.numel + (double)T1->numel);
    s1.bytes32 = 8.0 * ((double)L.numel + (double)psi.numel) + 4.0 * (double)T1->numel;
  }

  // ---- steps 2+3: T3 = h . T1 with h = W1.W2, per (a, y) sector pair
  Step hc, ha;
  hc.kind = StepKind::HCoef;
  hc.name = "mpo_coef";
  hc.constant = true;
  ha.kind = StepKind::HApply;
  ha.name = "mpo_apply";
  ha.has_alt = true;
  {
    const LegDesc& lw = L.legs[1];
    const LegDesc& lt1 = psi.legs[1];
    const LegDesc& lt2 = psi.legs[2];
    const LegDesc& ls1 = W1.legs[1];
    const LegDesc& ls2 = W2.legs[1];
    const LegDesc& lw3 = W2.legs[3];
    LegMap mw1(W1.legs[0]), ms1(W1.legs[1]), mt1(W1.legs[2]), mw2(W1.legs[3]);
    LegMap nw2(W2.legs[0]), ns2(W2.legs[1]), nt2(W2.legs[2]), nw3(W2.legs[3]);
    LegMap m1[4] = {mw1, ms1, mt1, mw2};
    LegMap m2[4] = {nw2, ns2, nt2, nw3};
    LegMap lwm(lw), lt1m(lt1), lt2m(lt2), ls1m(ls1), ls2m(ls2), lw3m(lw3);
    std::map<std::vector<int64_t>, int32_t> classes;
    const int nA = (int)psi.legs[0].q.size(), nY = (int)psi.legs[3].q.size();
    int32_t t[5];
    for (int ka = 0; ka < nA; ++ka)
      for (int ky = 0; ky < nY; ++ky) {
        std::vector<HPlane> ins, ins_alt, outs, outs_alt;
        std::vector<Step::FusedIn> fin;
        std::vector<int64_t> key;   // class key: input then output element triples
        for (int kw = 0; kw < (int)lw.q.size(); ++kw)
          for (int k1 = 0; k1 < (int)lt1.q.size(); ++k1)
            for (int k2 = 0; k2 < (int)lt2.q.size(); ++k2) {
              t[0] = ka; t[1] = kw; t[2] = k1; t[3] = k2; t[4] = ky;
              const int64_t b = T1->find(t);
              if (b < 0) continue;
              const int64_t gw = lw.g[kw], g1 = lt1.g[k1], g2 = lt2.g[k2], gy = psi.legs[3].g[ky];
              // the a' sector joining (a, w) to (t1, t2, y), and the block's
              // place in the merged T1 group of that sector
              // (blocks no pair reaches have a zero region of canonical shape)
              int64_t lb = -1, pb = -1;
              int kx = 0;
              if (t1zero[b] < 0) {
                for (; kx < (int)psi.legs[0].q.size(); ++kx) {
                  const int32_t lq[3] = {ka, kw, kx};
                  const int32_t pq[4] = {kx, k1, k2, ky};
                  lb = L.find(lq);
                  pb = psi.find(pq);
                  if (lb >= 0 && pb >= 0) break;
                }
                if (lb < 0 || pb < 0) fail(BST_E_INVALID, "internal: T1 block without a' sector");
              }
              for (int64_t c = 0; c < gw; ++c)
                for (int64_t e1 = 0; e1 < g1; ++e1)
                  for (int64_t e2 = 0; e2 < g2; ++e2) {
                    const int64_t in_blk = ((c * g1 + e1) * g2 + e2) * gy;
                    ins.push_back({T1->offset[b] + in_blk, gw * g1 * g2 * gy});
                    if (t1zero[b] >= 0) {
                      ins_alt.push_back({t1zero[b] + in_blk, gw * g1 * g2 * gy});
                      fin.push_back({0, 0, 0, 0, 0, 0});
                    } else {
                      const int64_t ld = t1m_ld[kx];
                      ins_alt.push_back({t1m_start[kx] + (Lg.grow[lb] + c) * ld + pcol[pb] +
                                             (e1 * g2 + e2) * gy,
                                         gw * ld});
                      // the GEMM of this T1 plane: L rows (grow + c + i gw) of
                      // the a' group against psi rows ((e1 g2 + e2) gy + j)
                      const int64_t K = psi.legs[0].g[kx], kp = pad32(K);
                      fin.push_back({Lg.gstart[kx] + (Lg.grow[lb] + c) * kp, Pp.off[pb] + (e1 * g2 + e2) * gy * kp,
                                     (int32_t)(gw * kp), (int32_t)kp, (int32_t)K, 0});
                    }
                    key.push_back(lwm.start[kw] + c);
                    key.push_back(lt1m.start[k1] + e1);
                    key.push_back(lt2m.start[k2] + e2);
                  }
            }
        key.push_back(-1);
        for (int k1 = 0; k1 < (int)ls1.q.size(); ++k1)
          for (int k2 = 0; k2 < (int)ls2.q.size(); ++k2)
            for (int kw = 0; kw < (int)lw3.q.size(); ++kw) {
              t[0] = ka; t[1] = k1; t[2] = k2; t[3] = kw; t[4] = ky;
              const int64_t b = T3->find(t);
              if (b < 0) continue;
              const int64_t g1 = ls1.g[k1], g2 = ls2.g[k2], gw = lw3.g[kw], gy = psi.legs[3].g[ky];
              // the output sector b joining (a, s1, s2) to (w3, b'): the
              // block's rows and columns in the merged T3 matrix of b
              int kb3 = 0;
              int64_t pb3 = -1, rb3 = -1;
              for (; kb3 < nB; ++kb3) {
                const int32_t pq[4] = {ka, k1, k2, kb3};
                const int32_t rq[3] = {kb3, kw, ky};
                pb3 = psi.find(pq);
                rb3 = R.find(rq);
                if (pb3 >= 0 && rb3 >= 0) break;
              }
              const bool read = pb3 >= 0 && rb3 >= 0;
              for (int64_t e1 = 0; e1 < g1; ++e1)
                for (int64_t e2 = 0; e2 < g2; ++e2)
                  for (int64_t c = 0; c < gw; ++c) {
                    outs.push_back({T3->offset[b] + ((e1 * g2 + e2) * gw + c) * gy, g1 * g2 * gw * gy});
                    if (read)
                      outs_alt.push_back({t3g[kb3] + (prow[pb3] + e1 * g2 + e2) * t3w[kb3] +
                                              rseg[rb3] + c * gy,
                                          g1 * g2 * t3w[kb3]});
                    else
                      outs_alt.push_back({t3sink, gy});
                    key.push_back(ls1m.start[k1] + e1);
                    key.push_back(ls2m.start[k2] + e2);
                    key.push_back(lw3m.start[kw] + c);
                  }
            }
        if (outs.empty()) continue;
        const int nin = (int)ins.size(), nout = (int)outs.size();
        int32_t cls;
        auto it = classes.find(key);
        if (it != classes.end()) {
          cls = it->second;
        } else {
          cls = (int32_t)classes.size();
          classes[key] = cls;
          // terms of coef[cls][o][i] = sum_w2 W1[w1,s1,t1,w2] W2[w2,s2,t2,w3]
          for (int o = 0; o < nout; ++o) {
            const int64_t S1 = key[3 * nin + 1 + 3 * o], S2 = key[3 * nin + 2 + 3 * o],
                          W3 = key[3 * nin + 3 + 3 * o];
            for (int i = 0; i < nin; ++i) {
              const int64_t Wl = key[3 * i], T1i = key[3 * i + 1], T2i = key[3 * i + 2];
              for (int64_t w2 = 0; w2 < (int64_t)mw2.sec.size(); ++w2) {
                const int64_t i1[4] = {Wl, S1, T1i, w2};
                const int64_t i2[4] = {w2, S2, T2i, W3};
                const int64_t o1 = elem_offset4(W1, m1, i1);
                if (o1 < 0) continue;
                const int64_t o2 = elem_offset4(W2, m2, i2);
                if (o2 < 0) continue;
                Step::RawTerm rt{};
                rt.cls = cls;
                rt.o = o;
                rt.i = i;
                rt.t.w1_buf = 1;
                rt.t.w2_buf = 2;
                rt.t.w1_off = o1;
                rt.t.w2_off = o2;
                hc.terms.push_back(rt);
              }
            }
          }
        }
        hc.nmax = std::max(hc.nmax, std::max(nin, nout));
        HTask task{};
        task.rows = (int32_t)psi.legs[0].g[ka];
        task.cols = (int32_t)psi.legs[3].g[ky];
        task.cls = cls;
        task.nin = nin;
        task.nout = nout;
        task.plane_begin = (int32_t)ha.planes.size();
        task.in_buf = 6;
        task.out_buf = 7;
        for (auto& q : ins) ha.planes.push_back(q);
        for (auto& q : outs) ha.planes.push_back(q);
        ha.tasks.push_back(task);
        ha.task_group.push_back(ka);
        ha.task_fin.push_back((int32_t)ha.fins.size());
        for (auto& f : fin) ha.fins.push_back(f);
        for (auto& q : ins_alt) ha.planes_alt.push_back(q);
        for (auto& q : outs_alt) ha.planes_alt.push_back(q);
        HTask ta = task;
        ta.out_buf = 11;
        ha.tasks_alt.push_back(ta);
      }
    hc.ncls = (int32_t)classes.size();
    ha.ncls = hc.ncls;
    ha.nmax = hc.nmax;
    // algorithmic flops of the two pairwise MPO contractions
    // step 2: T1[a,w1,t1,t2,y] . W1[w1,s1,t1,w2]; step 3: T2[a,t2,y,s1,w2] . W2[w2,s2,t2,w3]
    double f2 = 0, f3 = 0;
    int32_t wt[4];
    for (int64_t b = 0; b < T1->nblocks; ++b) {
      const int32_t* tb = T1->block_qn(b);
      for (int ks = 0; ks < (int)W1.legs[1].q.size(); ++ks)
        for (int kw2 = 0; kw2 < (int)W1.legs[3].q.size(); ++kw2) {
          wt[0] = tb[1]; wt[1] = ks; wt[2] = tb[2]; wt[3] = kw2;
          if (W1.find(wt) < 0) continue;
          f2 += 2.0 * (double)T1->block_size(b) * (double)(W1.legs[1].g[ks] * W1.legs[3].g[kw2]);
        }
    }
    auto T2 = make_tensor({lab(psi.legs[0], "a"), lab(psi.legs[2], "t2"), lab(psi.legs[3], "y"),
                           lab(W1.legs[1], "s1"), lab(W1.legs[3], "w2")});
    for (int64_t b = 0; b < T2->nblocks; ++b) {
      const int32_t* tb = T2->block_qn(b);
      for (int ks = 0; ks < (int)W2.legs[1].q.size(); ++ks)
        for (int kw3 = 0; kw3 < (int)W2.legs[3].q.size(); ++kw3) {
          wt[0] = tb[4]; wt[1] = ks; wt[2] = tb[1]; wt[3] = kw3;
          if (W2.find(wt) < 0) continue;
          f3 += 2.0 * (double)T2->block_size(b) * (double)(W2.legs[1].g[ks] * W2.legs[3].g[kw3]);
        }
    }
    ha.flops = f2 + f3;
    ha.bytes = 8.0 * ((double)T1->numel + (double)T3->numel);
    ha.bytes32 = 4.0 * ((double)T1->numel + (double)T3->numel);
  }

  // ---- step 4: out[(a s1 s2) x b] = sum_(w3,y) T3[(a s1 s2) x (w3 y)] R[b x (w3 y)]^T
  Step s4;
  s4.kind = StepKind::Gemm;
  s4.name = "gemm_T3_R";
  s4.ta = Elem::Inter;
  s4.transb = true;
  s4.has_alt = true;
  s4.writes_out = true;
  {
    const int nW = (int)W2.legs[3].q.size(), nY = (int)psi.legs[3].q.size();
    int32_t tt[5], rt[3];
    for (int64_t cb = 0; cb < psi.nblocks; ++cb) {
      const int32_t* t = psi.block_qn(cb);
      const int64_t* sh = psi.block_shape(cb);
      GemmProb p{};
      const int64_t M = sh[0] * sh[1] * sh[2], N = sh[3];
      p.c_off = psi.offset[cb];
      p.c_buf = 5;
      p.M = (int32_t)M;
      p.N = (int32_t)N;
      p.ldc = (int32_t)N;
      p.seg_begin = (int32_t)s4.segs.size();
      for (int kw = 0; kw < nW; ++kw)
        for (int ky = 0; ky < nY; ++ky) {
          tt[0] = t[0]; tt[1] = t[1]; tt[2] = t[2]; tt[3] = kw; tt[4] = ky;
          rt[0] = t[3]; rt[1] = kw; rt[2] = ky;
          const int64_t ab = T3->find(tt), bb = R.find(rt);
          if (ab < 0 || bb < 0) continue;
          const int64_t K = W2.legs[3].g[kw] * psi.legs[3].g[ky];
          GemmSeg g{};
          g.a_off = T3->offset[ab];
          g.a_buf = 7;
          g.b_off = R.offset[bb];
          g.b_buf = 3;
          g.K = (int32_t)K;
          g.lda = (int32_t)K;
          g.ldb = (int32_t)K;
          s4.segs.push_back(g);
          s4.flops += 2.0 * (double)M * (double)N * (double)K;
        }
      p.seg_count = (int32_t)s4.segs.size() - p.seg_begin;
      s4.probs.push_back(p);
    }
    // plane variant: one problem per output sector b over the merged T3
    // rows; each row is written to its psi block through the row map
    for (int kb = 0; kb < nB; ++kb) {
      if (t3m[kb] == 0) continue;
      if (t3m[kb] > 0x7FFFFFFF) fail(BST_E_INVALID, "sector group too large");
      const int64_t Nb = psi.legs[3].g[kb];
      GemmProb p{};
      p.c_off = 0;
      p.c_buf = 5;
      p.M = (int32_t)t3m[kb];
      p.N = (int32_t)Nb;
      p.ldc = (int32_t)Nb;
      p.seg_begin = (int32_t)s4.segs_alt.size();
      p.rowmap1 = (int32_t)s4.rowmap.size() + 1;
      for (int64_t b = 0; b < psi.nblocks; ++b) {
        if (psi.block_qn(b)[3] != kb) continue;
        const int64_t rows = psi.block_shape(b)[0] * psi.block_shape(b)[1] * psi.block_shape(b)[2];
        for (int64_t r = 0; r < rows; ++r) s4.rowmap.push_back(psi.offset[b] + r * Nb);
      }
      for (int64_t rb = 0; rb < R.nblocks; ++rb) {
        if (R.block_qn(rb)[0] != kb) continue;
        GemmSeg h{};
        h.K = (int32_t)(R.block_shape(rb)[1] * R.block_shape(rb)[2]);
        h.a_off = t3g[kb] + rseg[rb];
        h.a_buf = 11;
        h.lda = (int32_t)t3w[kb];
        h.b_off = Rp.off[rb];
        h.b_buf = 9;
        h.ldb = (int32_t)Rp.ld[rb];
        s4.segs_alt.push_back(h);
      }
      p.seg_count = (int32_t)s4.segs_alt.size() - p.seg_begin;
      s4.probs_alt.push_back(p);
    }
    if ((int64_t)s4.rowmap.size() > 0x7FFFFFFF) fail(BST_E_INVALID, "row map too large");
    s4.bytes = 8.0 * ((double)T3->numel + (double)R.numel + (double)psi.numel);
    s4.bytes32 = 4.0 * (double)T3->numel + 8.0 * ((double)R.numel + (double)psi.numel);
  }
  P.steps.push_back(std::move(hc));
  P.steps.push_back(std::move(spL));
  P.steps.push_back(std::move(spR));
  P.steps.push_back(std::move(spP));
  P.steps.push_back(std::move(s1));
  P.steps.push_back(std::move(ha));
  P.steps.push_back(std::move(s4));
}

// Merges n H_eff plans: slot s of plan i becomes base_i + s.
static void heff_batch(const std::vector<const PlanData*>& subs, PlanData& P) {
  P.kind = 3;
  P.nslots = 0;
  int32_t cls_base = 0;
  for (size_t i = 0; i < subs.size(); ++i) {
    const PlanData& S = *subs[i];
    if (S.kind != 2) fail(BST_E_INVALID, "batch members must be H_eff plans");
    const int32_t base = P.nslots;
    for (auto s : S.in_slots) P.in_slots.push_back(base + s);
    for (auto s : S.out_slots) P.out_slots.push_back(base + s);
    for (auto n : S.in_numel) P.in_numel.push_back(n);
    for (auto n : S.out_numel) P.out_numel.push_back(n);
    for (auto ib : S.internals) P.internals.push_back({base + ib.slot, ib.bytes, 0});
    if (P.steps.empty()) {
      for (const auto& st : S.steps) {
        Step e;
        e.kind = st.kind;
        e.name = st.name;
        e.ta = st.ta;
        e.tc = st.tc;
        e.transb = st.transb;
        e.th = st.th;
        e.has_alt = st.has_alt;
        e.constant = st.constant;
        P.steps.push_back(std::move(e));
      }
    }
    if (P.steps.size() != S.steps.size()) fail(BST_E_INVALID, "inconsistent batch members");
    for (size_t k = 0; k < S.steps.size(); ++k) {
      const Step& a = S.steps[k];
      Step& b = P.steps[k];
      b.flops += a.flops;
      b.bytes += a.bytes;
      b.bytes32 += a.bytes32;
      if (a.kind == StepKind::Gemm) {
        const int32_t sb = (int32_t)b.segs.size();
        for (auto g : a.segs) {
          g.a_buf += base;
          g.b_buf += base;
          b.segs.push_back(g);
        }
        for (auto p : a.probs) {
          p.c_buf += base;
          p.seg_begin += sb;
          b.probs.push_back(p);
        }
        const int32_t sba = (int32_t)b.segs_alt.size();
        for (auto g : a.segs_alt) {
          g.a_buf += base;
          g.b_buf += base;
          b.segs_alt.push_back(g);
        }
        const int32_t rmb = (int32_t)b.rowmap.size();
        for (auto r : a.rowmap) b.rowmap.push_back(r);
        for (auto p : a.probs_alt) {
          p.c_buf += base;
          p.seg_begin += sba;
          if (p.rowmap1 > 0) p.rowmap1 += rmb;
          b.probs_alt.push_back(p);
        }
      } else if (a.kind == StepKind::HCoef) {
        for (auto rt : a.terms) {
          rt.cls += cls_base;
          rt.t.w1_buf += base;
          rt.t.w2_buf += base;
          b.terms.push_back(rt);
        }
        b.ncls += a.ncls;
        b.nmax = std::max(b.nmax, a.nmax);
      } else if (a.kind == StepKind::HApply) {
        const int32_t pb = (int32_t)b.planes.size();
        // task groups stay distinct between members
        const int32_t gb =
            b.task_group.empty() ? 0 : *std::max_element(b.task_group.begin(), b.task_group.end()) + 1;
        for (auto g : a.task_group) b.task_group.push_back(g + gb);
        for (auto q : a.planes) b.planes.push_back(q);
        for (auto t : a.tasks) {
          t.cls += cls_base;
          t.plane_begin += pb;
          t.in_buf += base;
          t.out_buf += base;
          b.tasks.push_back(t);
        }
        const int32_t pba = (int32_t)b.planes_alt.size();
        for (auto q : a.planes_alt) b.planes_alt.push_back(q);
        for (auto t : a.tasks_alt) {
          t.cls += cls_base;
          t.plane_begin += pba;
          t.in_buf += base;
          t.out_buf += base;
          b.tasks_alt.push_back(t);
        }
        b.ncls += a.ncls;
        b.nmax = std::max(b.nmax, a.nmax);
      } else if (a.kind == StepKind::Split) {
        const int32_t jb = (int32_t)b.sjobs.size();
        for (auto j : a.sjobs) {
          j.in_buf += base;
          j.out_buf += base;
          b.sjobs.push_back(j);
        }
        for (auto w : a.swork) {
          w.job += jb;
          b.swork.push_back(w);
        }
      }
    }
    // class ids advance by the member's class count
    for (const auto& st : S.steps)
      if (st.kind == StepKind::HCoef) cls_base += st.ncls;
    P.nslots += S.nslots;
    P.psi_numel += S.psi_numel;
    P.has_planes = (i == 0 ? S.has_planes : (P.has_planes && S.has_planes));
  }
}

// ------------------------------------------------------------------------
// Finalize: device tables laid out in one blob, workspace layout
// ------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
static size_t put(std::vector<uint8_t>& blob, const std::vector<T>& v) {
  size_t off = align256(blob.size());
  blob.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

static int round_nmax(int n) {
  if (n <= 8) return 8;
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  fail(BST_E_INVALID, "two-site MPO apply needs more than 64 channels per sector pair");
}

// Tiles of a grouped GEMM for one tile shape, in dispatch order.
//
// Workgroups go to the 8 XCDs round-robin by linear id, and each XCD has its
// own L2.  The tiles of one problem share their A row panels and B column
// panels, so whole problems are bin-packed onto XCDs (largest cost first,
// each to the least loaded XCD), each XCD's tiles are ordered by cost with a
// problem's tiles kept together, and the eight lists are interleaved so that
// linear id 8*pos + x is tile pos of XCD x.  Short lists are padded with
// empty tiles (prob = -1) that exit at once.
constexpr int kXcds = 8;

static std::vector<GemmTile> make_tiles(const std::vector<GemmProb>& probs,
                                        const std::vector<GemmSeg>& segs, int bm, int bn) {
  struct Prob {
    double cost;
    int32_t idx;
  };
  std::vector<Prob> pr;
  for (size_t pi = 0; pi < probs.size(); ++pi) {
    const auto& p = probs[pi];
    int64_t k = 0;
    for (int s = 0; s < p.seg_count; ++s) k += segs[p.seg_begin + s].K;
    const double ntile = (double)((p.M + bm - 1) / bm) * (double)((p.N + bn - 1) / bn);
    pr.push_back({ntile * (double)(k + 16), (int32_t)pi});
  }
  std::stable_sort(pr.begin(), pr.end(), [](const Prob& a, const Prob& b) { return a.cost > b.cost; });
  std::vector<std::vector<GemmTile>> bins(kXcds);
  std::vector<double> load(kXcds, 0.0);
  for (const auto& q : pr) {
    int x = 0;
    for (int i = 1; i < kXcds; ++i)
      if (load[i] < load[x]) x = i;
    load[x] += q.cost;
    const auto& p = probs[q.idx];
    for (int m0 = 0; m0 < p.M; m0 += bm)
      for (int n0 = 0; n0 < p.N; n0 += bn) bins[x].push_back({q.idx, m0, n0, 0});
  }
  size_t longest = 0;
  for (auto& b : bins) longest = std::max(longest, b.size());
  std::vector<GemmTile> out;
  out.reserve(longest * kXcds);
  for (size_t pos = 0; pos < longest; ++pos)
    for (int x = 0; x < kXcds; ++x)
      out.push_back(pos < bins[x].size() ? bins[x][pos] : GemmTile{-1, 0, 0, 0});
  // drop trailing empty tiles
  while (!out.empty() && out.back().prob < 0) out.pop_back();
  return out;
}

// k-step schedule of the pipelined plane kernel for one tile shape.  The
// problems go to the XCDs as in make_tiles; each XCD's tiles, in that
// order, go one by one to the least loaded of the XCD's workgroups
// (workgroup w runs on XCD w % 8); a workgroup's tiles become consecutive
// k-step records.  ok stays false if an operand offset or row stride is not
// a multiple of 8 positions (whole 16-byte pieces) or a table slot does not
// fit the record.
//
// np = 1 (float64 operands): 16-deep steps whose "chunks" are 16-byte
// pieces of two elements.
static Step::StreamList make_stream(std::vector<uint8_t>& blob, const Step& st, int np, const TileShape& sh) {
  Step::StreamList L;
  const auto& probs = st.probs_alt;
  const auto& segs = st.segs_alt;
  const int bm = sh.bm, bn = sh.bn;
  // k elements per step and per chunk, chunks per step
  const int64_t kdeep = np == 1 ? 16 : 32, kchunk = np == 1 ? 2 : 8, nchunk = kdeep / kchunk;
  auto padc = [&](int64_t K) { return (K + kchunk - 1) / kchunk * kchunk; };
  if (bm > 256 || bn > 256) return L;   // row / column counts are stored in a byte
  for (const auto& g : segs) {
    if (g.K <= 0) continue;
    if (g.a_off % 8 || g.b_off % 8 || g.lda % 8 || g.ldb % 8) return L;
    if (g.a_buf < 0 || g.a_buf > 0xFFFF || g.b_buf < 0 || g.b_buf > 0xFFFF) return L;
  }
  for (const auto& p : probs)
    if (p.c_buf < 0 || p.c_buf > 0xFFFF) return L;
  auto ksteps = [&](const GemmProb& p) {
    int64_t k = 0;
    for (int q = 0; q < p.seg_count; ++q) {
      const int64_t K = segs[p.seg_begin + q].K;
      if (K > 0) k += (padc(K) + kdeep - 1) / kdeep;
    }
    return std::max<int64_t>(k, 1);
  };
  // problems to XCDs: largest first, each to the least loaded
  struct Prob {
    double cost;
    int32_t idx;
  };
  std::vector<Prob> pr;
  for (size_t pi = 0; pi < probs.size(); ++pi) {
    const auto& p = probs[pi];
    const double nt = (double)((p.M + bm - 1) / bm) * (double)((p.N + bn - 1) / bn);
    pr.push_back({nt * (double)(ksteps(p) + 2), (int32_t)pi});
  }
  std::stable_sort(pr.begin(), pr.end(), [](const Prob& a, const Prob& b) { return a.cost > b.cost; });
  std::vector<double> xload(kXcds, 0.0);
  std::vector<std::vector<GemmTile>> bins(kXcds);
  for (const auto& q : pr) {
    int x = 0;
    for (int i = 1; i < kXcds; ++i)
      if (xload[i] < xload[x]) x = i;
    xload[x] += q.cost;
    const auto& p = probs[q.idx];
    for (int m0 = 0; m0 < p.M; m0 += bm)
      for (int n0 = 0; n0 < p.N; n0 += bn) bins[x].push_back({q.idx, m0, n0, 0});
  }
  const int64_t nwg = (int64_t)kStreamCUs * stream_wgs_per_cu(np, bm, bn, sh.stages);
  std::vector<std::vector<GemmTile>> per(nwg);
  std::vector<int64_t> wload(nwg, 0);
  for (int x = 0; x < kXcds; ++x)
    for (const auto& t : bins[x]) {
      int64_t w = x;
      for (int64_t c = x + kXcds; c < nwg; c += kXcds)
        if (wload[c] < wload[w]) w = c;
      per[w].push_back(t);
      wload[w] += ksteps(probs[t.prob]) + 2;
    }
  std::vector<KStep> recs;
  std::vector<int64_t> begin((size_t)nwg + 1, 0), rowtab;
  for (int64_t w = 0; w < nwg; ++w) {
    begin[w] = (int64_t)recs.size();
    for (const auto& t : per[w]) {
      const GemmProb& p = probs[t.prob];
      KStep base{};
      const int rows = std::min(bm, p.M - t.m0), cols = std::min(bn, p.N - t.n0);
      base.rows1 = (uint8_t)(rows - 1);
      base.cols1 = (uint8_t)(cols - 1);
      base.c_buf = (uint16_t)p.c_buf;
      base.kval = (uint8_t)kchunk;
      if (p.rowmap1 > 0) {
        base.flags = kStepRowmap;
        base.c = (int64_t)rowtab.size();
        for (int r = 0; r < bm; ++r)
          rowtab.push_back(r < rows ? st.rowmap[(size_t)(p.rowmap1 - 1 + t.m0 + r)] + t.n0 : -1);
      } else {
        base.c = p.c_off + (int64_t)t.m0 * p.ldc + t.n0;
        base.ldc = p.ldc;
      }
      const size_t first = recs.size();
      for (int q = 0; q < p.seg_count; ++q) {
        const GemmSeg& g = segs[p.seg_begin + q];
        if (g.K <= 0) continue;
        const int64_t K8 = padc(g.K);
        for (int64_t lk = 0; lk < K8; lk += kdeep) {
          KStep k = base;
          k.a = g.a_off + (int64_t)t.m0 * g.lda + lk;
          k.b = g.b_off + (int64_t)t.n0 * g.ldb + lk;
          k.lda = g.lda;
          k.ldb = g.ldb;
          k.a_buf = (uint16_t)g.a_buf;
          k.b_buf = (uint16_t)g.b_buf;
          k.kch = (uint8_t)std::min<int64_t>(nchunk, (K8 - lk) / kchunk);
          k.kval = (uint8_t)((lk + kchunk * k.kch == K8 && g.K % kchunk) ? g.K % kchunk : kchunk);
          recs.push_back(k);
        }
      }
      if (recs.size() == first) {   // no k-steps: one step of zeros writes the tile
        KStep k = base;
        k.kch = 0;
        k.a_buf = k.b_buf = (uint16_t)p.c_buf;
        recs.push_back(k);
      }
      recs[first].flags |= kStepFirst;
      recs.back().flags |= kStepLast;
    }
  }
  begin[nwg] = (int64_t)recs.size();
  recs.resize(recs.size() + kStepBatch, KStep{});   // batches read whole
  rowtab.push_back(-1);
  rowtab.push_back(-1);
  L.steps_off = put(blob, recs);
  L.begin_off = put(blob, begin);
  L.rows_off = put(blob, rowtab);
  L.nwg = nwg;
  L.ok = true;
  return L;
}

// k-step schedule of the fused L.psi + MPO kernel (two bfloat16 planes):
// 64 x 64 tiles of every task of tasks_alt, each tile's records channel by
// channel (the k-steps of input p's GEMM, the last flagged kStepPlaneEnd).
// Tiles go to the XCDs by a sector (as the MPO work items: tasks of one a
// share L rows, psi blocks and T3 rows), largest a first to the least
// loaded XCD; there, by first row, each to the least loaded workgroup.  ok
// stays false unless every task fits the kernel (nmax <= 16 inputs and
// outputs, 16-byte aligned operands).
static Step::StreamList make_fused(std::vector<uint8_t>& blob, const Step& st, int nmax) {
  Step::StreamList L;
  constexpr int bm = 64, bn = 64;
  const int64_t kdeep = 32, kchunk = 8, nchunk = 4;
  auto padc = [&](int64_t K) { return (K + kchunk - 1) / kchunk * kchunk; };
  if (st.fins.empty() || st.tasks_alt.size() != st.task_fin.size() || nmax > 16) return L;
  for (size_t ti = 0; ti < st.tasks_alt.size(); ++ti) {
    const HTask& t = st.tasks_alt[ti];
    if (t.nin > nmax || t.nout > nmax || t.nin > 255) return L;
    for (int p = 0; p < t.nin; ++p) {
      const auto& f = st.fins[(size_t)st.task_fin[ti] + p];
      if (f.K > 0 && (f.a_off % 8 || f.b_off % 8 || f.a_ld % 8 || f.b_ld % 8)) return L;
    }
  }
  struct Tile {
    int32_t task, m0, n0;
    int64_t steps;
  };
  auto tile_steps = [&](int32_t ti) {
    int64_t k = 0;
    const HTask& t = st.tasks_alt[ti];
    for (int p = 0; p < t.nin; ++p) {
      const int32_t K = st.fins[(size_t)st.task_fin[ti] + p].K;
      if (K > 0) k += (padc(K) + kdeep - 1) / kdeep;
    }
    return std::max<int64_t>(k, 1);
  };
  std::map<int32_t, std::vector<Tile>> groups;
  std::map<int32_t, int64_t> gcost;
  for (size_t ti = 0; ti < st.tasks_alt.size(); ++ti) {
    const HTask& t = st.tasks_alt[ti];
    const int32_t g = ti < st.task_group.size() ? st.task_group[ti] : 0;
    const int64_t ks = tile_steps((int32_t)ti);
    for (int m0 = 0; m0 < t.rows; m0 += bm)
      for (int n0 = 0; n0 < t.cols; n0 += bn) {
        groups[g].push_back({(int32_t)ti, m0, n0, ks + 2});
        gcost[g] += ks + 2;
      }
  }
  std::vector<std::pair<int64_t, int32_t>> order;
  for (auto& kv : gcost) order.push_back({kv.second, kv.first});
  std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<std::vector<Tile>> bins(kXcds);
  std::vector<int64_t> xload(kXcds, 0);
  for (const auto& o : order) {
    int x = 0;
    for (int i = 1; i < kXcds; ++i)
      if (xload[i] < xload[x]) x = i;
    xload[x] += o.first;
    auto& tl = groups[o.second];
    std::stable_sort(tl.begin(), tl.end(), [](const Tile& a, const Tile& b) { return a.m0 < b.m0; });
    bins[x].insert(bins[x].end(), tl.begin(), tl.end());
  }
  // one workgroup of 8 waves per CU (16 outputs: 194 VGPRs), two with 8
  const int64_t nwg = (int64_t)kStreamCUs * (nmax <= 8 ? 2 : 1);
  std::vector<std::vector<Tile>> per(nwg);
  std::vector<int64_t> wload(nwg, 0);
  for (int x = 0; x < kXcds; ++x)
    for (const auto& t : bins[x]) {
      int64_t w = x;
      for (int64_t c = x + kXcds; c < nwg; c += kXcds)
        if (wload[c] < wload[w]) w = c;
      per[w].push_back(t);
      wload[w] += t.steps;
    }
  std::vector<KStep> recs;
  std::vector<int64_t> begin((size_t)nwg + 1, 0);
  for (int64_t w = 0; w < nwg; ++w) {
    begin[w] = (int64_t)recs.size();
    for (const auto& tl : per[w]) {
      const HTask& t = st.tasks_alt[tl.task];
      KStep base{};
      base.rows1 = (uint8_t)(std::min(bm, t.rows - tl.m0) - 1);
      base.cols1 = (uint8_t)(std::min(bn, t.cols - tl.n0) - 1);
      base.c_buf = (uint16_t)t.nout;
      base.c = (int64_t)((uint64_t)(uint32_t)(t.cls * nmax * nmax) |
                         ((uint64_t)(uint32_t)(t.plane_begin + t.nin) << 32));
      base.ldc = (int32_t)((uint32_t)tl.m0 | ((uint32_t)tl.n0 << 16));
      base.a_buf = 8;
      base.b_buf = 10;
      base.kval = (uint8_t)kchunk;
      const size_t first = recs.size();
      for (int p = 0; p < t.nin; ++p) {
        const auto& f = st.fins[(size_t)st.task_fin[tl.task] + p];
        if (f.K <= 0) continue;
        const int64_t K8 = padc(f.K);
        for (int64_t lk = 0; lk < K8; lk += kdeep) {
          KStep k = base;
          k.a = f.a_off + (int64_t)tl.m0 * f.a_ld + lk;
          k.b = f.b_off + (int64_t)tl.n0 * f.b_ld + lk;
          k.lda = f.a_ld;
          k.ldb = f.b_ld;
          k.pad = (uint8_t)p;
          k.kch = (uint8_t)std::min<int64_t>(nchunk, (K8 - lk) / kchunk);
          k.kval = (uint8_t)((lk + kchunk * k.kch == K8 && f.K % kchunk) ? f.K % kchunk : kchunk);
          recs.push_back(k);
        }
        recs.back().flags |= kStepPlaneEnd;
      }
      if (recs.size() == first) {   // every input zero: one step of zeros writes the tile
        KStep k = base;
        k.kch = 0;
        k.pad = 0;
        k.flags = kStepPlaneEnd;
        recs.push_back(k);
      }
      recs[first].flags |= kStepFirst;
      recs.back().flags |= kStepLast;
    }
  }
  begin[nwg] = (int64_t)recs.size();
  recs.resize(recs.size() + kStepBatch, KStep{});
  L.steps_off = put(blob, recs);
  L.begin_off = put(blob, begin);
  L.nwg = nwg;
  L.ok = true;
  return L;
}

int default_tile(const Step& st, bst_precision form) {
  auto it = st.tile_choice.find((int)form);
  if (it != st.tile_choice.end()) return it->second;
  // float64 / float32: the LDS-staged 64x64 kernel
  if (form == BST_FP64 || form == BST_FP32) return 5;
  // on-the-fly split forms: 64x64 unless most problems are small
  const auto& shapes = gemm_tile_shapes(form);
  double avg = 0;
  for (auto& p : st.probs) avg += std::min(p.M, p.N);
  if (!st.probs.empty()) avg /= (double)st.probs.size();
  const int want = avg < 48 ? 32 : 64;
  for (size_t i = 0; i < shapes.size(); ++i)
    if (shapes[i].bm == want && shapes[i].bn == want) return (int)i;
  return 0;
}

void finalize(PlanData& P) {
  P.blob.clear();
  P.coef_entries = 0;
  P.fused_ok = false;
  for (auto& st : P.steps) {
    switch (st.kind) {
      case StepKind::Gemm: {
        st.off0 = put(P.blob, st.probs);
        st.off1 = put(P.blob, st.segs);
        st.tile_lists.clear();
        st.tile_lists_alt.clear();
        for (int f = 0; f < 4; ++f)
          for (const auto& sh : gemm_tile_shapes((bst_precision)f)) {
            auto key = std::make_pair(sh.bm, sh.bn);
            if (st.tile_lists.count(key)) continue;
            auto tl = make_tiles(st.probs, st.segs, sh.bm, sh.bn);
            st.tile_lists[key] = {put(P.blob, tl), (int64_t)tl.size()};
          }
        if (st.has_alt) {
          st.off2 = put(P.blob, st.segs_alt);
          st.off3 = put(P.blob, st.probs_alt);
          st.off5 = put(P.blob, st.rowmap);
          st.streams_alt.clear();
          for (int np = 1; np <= 3; ++np) {
            const auto& shapes = gemm_planes_shapes(np);
            for (size_t i = 0; i < shapes.size(); ++i) {
              const auto& sh = shapes[i];
              if (sh.direct == 3) {
                st.streams_alt[np * 64 + (int)i] = make_stream(P.blob, st, np, sh);
                continue;
              }
              auto key = std::make_pair(sh.bm, sh.bn);
              if (st.tile_lists_alt.count(key)) continue;
              auto tl = make_tiles(st.probs_alt, st.segs_alt, sh.bm, sh.bn);
              st.tile_lists_alt[key] = {put(P.blob, tl), (int64_t)tl.size()};
            }
          }
        }
        break;
      }
      case StepKind::Expand:
        st.off0 = put(P.blob, st.xjobs);
        st.off1 = put(P.blob, st.xwork);
        st.n0 = (int64_t)st.xwork.size();
        break;
      case StepKind::Permute:
        st.off0 = put(P.blob, st.jobs);
        st.off1 = put(P.blob, st.pwork);
        st.n0 = (int64_t)st.pwork.size();
        break;
      case StepKind::HCoef: {
        const int nm = st.terms.empty() && st.ncls == 0 ? 8 : round_nmax(st.nmax);
        st.nmax = nm;
        const int64_t nent = (int64_t)st.ncls * nm * nm;
        std::vector<std::vector<HTerm>> per(nent);
        for (auto& rt : st.terms) per[((int64_t)rt.cls * nm + rt.o) * nm + rt.i].push_back(rt.t);
        std::vector<HTerm> flat;
        std::vector<int32_t> begin(nent + 1, 0);
        for (int64_t e = 0; e < nent; ++e) {
          begin[e] = (int32_t)flat.size();
          for (auto& t : per[e]) flat.push_back(t);
        }
        begin[nent] = (int32_t)flat.size();
        st.off0 = put(P.blob, flat);
        st.off1 = put(P.blob, begin);
        st.n0 = nent;
        P.coef_entries = (int32_t)std::max<int64_t>(P.coef_entries, nent);
        break;
      }
      case StepKind::HApply: {
        st.nmax = st.ncls == 0 ? 8 : round_nmax(st.nmax);
        // largest element index of every plane, times 3 (plane interleave)
        // plus a chunk, times the widest element (8 bytes), below 2^32
        auto fit32 = [](const std::vector<HTask>& ts, const std::vector<HPlane>& ps) {
          for (const auto& t : ts)
            for (int32_t q = 0; q < t.nin + t.nout; ++q) {
              const HPlane& pl = ps[(size_t)t.plane_begin + q];
              if (pl.off < 0 || pl.rowstride < 0) return false;
              const int64_t last = pl.off + (int64_t)(t.rows > 0 ? t.rows - 1 : 0) * pl.rowstride +
                                   (t.cols > 0 ? t.cols - 1 : 0);
              if ((last + 8) * 3 * 8 >= ((int64_t)1 << 32)) return false;
            }
          return true;
        };
        // BST_MPO_INDEX64 (any value) keeps 64-bit indexing even where 32
        // bits would do, so that path can be exercised on small operators
        const bool force64 = std::getenv("BST_MPO_INDEX64") != nullptr;
        st.mpo_off32 = !force64 && fit32(st.tasks, st.planes);
        st.mpo_off32_alt = !force64 && st.has_alt && fit32(st.tasks_alt, st.planes_alt);
        // Work items of 256 sites, in two orders.  Task by task (work):
        // consecutive items spread over all XCDs.  Grouped (work_grouped,
        // used when the apply writes bfloat16 planes): the tasks of one a
        // sector read the same T1 rows and write the same T3 rows, each its
        // own column segment, so lines at segment ends are shared between
        // them.  Each XCD has its own L2 and workgroups go to the XCDs
        // round-robin, so the items of one a sector go to one XCD (sectors
        // by size, largest first, each to the least loaded XCD), ordered
        // there by first row, and the eight lists are interleaved
        // (workgroup 8 pos + x runs item pos of XCD x).  Short lists end in
        // empty items (site0 past the task).  With float64 outputs the
        // grouped order measured slower (87 -> 90 us per apply at chi = 4096).
        std::vector<HWork> work, wgrp;
        for (size_t ti = 0; ti < st.tasks.size(); ++ti) {
          const int64_t sites = (int64_t)st.tasks[ti].rows * st.tasks[ti].cols;
          for (int64_t s0 = 0; s0 < sites; s0 += 256) work.push_back({(int32_t)ti, (int32_t)s0});
        }
        {
          struct Item {
            int32_t task, s0, row0;
          };
          std::map<int32_t, std::vector<Item>> groups;
          for (size_t ti = 0; ti < st.tasks.size(); ++ti) {
            const int64_t sites = (int64_t)st.tasks[ti].rows * st.tasks[ti].cols;
            const int32_t g = ti < st.task_group.size() ? st.task_group[ti] : 0;
            for (int64_t s0 = 0; s0 < sites; s0 += 256)
              groups[g].push_back({(int32_t)ti, (int32_t)s0, (int32_t)(s0 / std::max(st.tasks[ti].cols, 1))});
          }
          std::vector<std::pair<size_t, int32_t>> order;
          for (auto& kv : groups) order.push_back({kv.second.size(), kv.first});
          std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
          std::vector<std::vector<Item>> bins(kXcds);
          for (const auto& o : order) {
            int x = 0;
            for (int i = 1; i < kXcds; ++i)
              if (bins[i].size() < bins[x].size()) x = i;
            auto& items = groups[o.second];
            std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.row0 < b.row0; });
            bins[x].insert(bins[x].end(), items.begin(), items.end());
          }
          size_t longest = 0;
          for (auto& b : bins) longest = std::max(longest, b.size());
          const int32_t empty_s0 = st.tasks.empty() ? 0 : st.tasks[0].rows * st.tasks[0].cols;
          for (size_t pos = 0; pos < longest; ++pos)
            for (int x = 0; x < kXcds; ++x)
              wgrp.push_back(pos < bins[x].size() ? HWork{bins[x][pos].task, bins[x][pos].s0}
                                                  : HWork{0, empty_s0});
          while (!wgrp.empty() && wgrp.back().task == 0 && wgrp.back().site0 == empty_s0 && empty_s0 > 0)
            wgrp.pop_back();
        }
        st.off0 = put(P.blob, st.tasks);
        st.off1 = put(P.blob, st.planes);
        st.off2 = put(P.blob, work);
        st.n0 = (int64_t)work.size();
        st.off5 = put(P.blob, wgrp);
        st.n1 = (int64_t)wgrp.size();
        if (st.has_alt) {
          st.off3 = put(P.blob, st.tasks_alt);
          st.off4 = put(P.blob, st.planes_alt);
          // the fused kernel copies nmax output planes per tile: spare records
          std::vector<HPlane> pl = st.planes_alt;
          pl.resize(pl.size() + (size_t)st.nmax, HPlane{0, 0});
          st.fused_planes_off = put(P.blob, pl);
          st.fused = make_fused(P.blob, st, st.nmax);
          if (st.fused.ok) P.fused_ok = true;
        }
        break;
      }
      case StepKind::Split:
      {
        std::vector<SplitItem> items;
        items.reserve(st.swork.size());
        for (const auto& w : st.swork) {
          const SplitJob& j = st.sjobs[w.job];
          items.push_back({j.in_off, j.out_off, j.in_buf, j.out_buf, j.rows, j.cols, j.out_ld, j.transpose, w.r0,
                           w.c0});
        }
        st.off0 = put(P.blob, items);
        st.n0 = (int64_t)items.size();
      }
        break;
    }
  }
  size_t off = 0;
  P.ws_ptr_off = off;
  off = align256(off + sizeof(void*) * (size_t)std::max(P.nslots, 1));
  P.ws_blob_off = off;
  off = align256(off + P.blob.size());
  P.ws_coef64_off = off;
  off = align256(off + sizeof(double) * (size_t)std::max(P.coef_entries, 1));
  P.ws_coef32_off = off;
  off = align256(off + sizeof(float) * (size_t)std::max(P.coef_entries, 1));
  P.ws_cnt_off = off;
  off = align256(off + sizeof(int32_t) * (size_t)std::max(P.coef_entries, 1));
  P.ws_idx_off = off;
  off = align256(off + sizeof(int32_t) * (size_t)std::max(P.coef_entries, 1));
  P.ws_val64_off = off;
  off = align256(off + sizeof(double) * (size_t)std::max(P.coef_entries, 1));
  P.ws_val32_off = off;
  off = align256(off + sizeof(float) * (size_t)std::max(P.coef_entries, 1));
  for (auto& ib : P.internals) {
    ib.ws_off = off;
    off = align256(off + std::max<size_t>(ib.bytes, 8));
  }
  P.ws_bytes = off;
  P.f64_panels = P.has_planes;
  for (const auto& st : P.steps) {
    if (st.kind != StepKind::Gemm || !st.has_alt) continue;
    bool any = false;
    for (const auto& kv : st.streams_alt) any = any || (kv.first / 64 == 1 && kv.second.ok);
    P.f64_panels = P.f64_panels && any;
  }
  P.finalized = true;
  P.uploaded_ws = nullptr;
  P.last_ptrs.clear();
  P.id = g_plan_id++;
}

}  // namespace bst

using namespace bst;

static bst_plan* new_plan() { return new bst_plan; }

extern "C" {

bst_status bst_permute_plan(const bst_tensor* in, const char* const* new_order,
                            bst_tensor** out_meta, bst_plan** plan) {
  BST_TRY
  if (!in || !out_meta || !plan) fail(BST_E_INVALID, "null argument");
  *out_meta = nullptr;
  *plan = nullptr;
  const TensorDesc& T = *desc_of(in);
  if (T.rank() > 0 && !new_order) fail(BST_E_INVALID, "null label list");
  std::vector<int> perm;
  for (int i = 0; i < T.rank(); ++i) {
    if (!new_order[i]) fail(BST_E_LABEL, "null label");
    int k = T.label_index(new_order[i]);
    if (k < 0) fail(BST_E_LABEL, std::string("unknown label '") + new_order[i] + "'");
    if (std::find(perm.begin(), perm.end(), k) != perm.end())
      fail(BST_E_LABEL, std::string("label listed twice '") + new_order[i] + "'");
    perm.push_back(k);
  }
  auto out = permuted_desc(T, perm);
  auto* p = new_plan();
  PlanData& P = p->p;
  P.kind = 0;
  P.in_slots = {0};
  P.out_slots = {1};
  P.in_numel = {T.numel};
  P.out_numel = {out->numel};
  P.nslots = 2;
  Step st;
  st.kind = StepKind::Permute;
  st.name = "permute";
  add_permute_jobs(st, T, *out, perm, 0, 1);
  P.steps.push_back(std::move(st));
  finalize(P);
  *plan = p;
  *out_meta = wrap_tensor(std::move(out));
  BST_CATCH
}

bst_status bst_contract_plan(const bst_tensor* A, const bst_tensor* B, bst_precision prec,
                             bst_tensor** C_meta, bst_plan** plan) {
  BST_TRY
  if (!A || !B || !C_meta || !plan) fail(BST_E_INVALID, "null argument");
  *C_meta = nullptr;
  *plan = nullptr;
  if (prec < BST_FP64 || prec > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  std::unique_ptr<TensorDesc> C;
  auto* p = new_plan();
  try {
    contract_plan(*desc_of(A), *desc_of(B), p->p, C);
    p->p.prec = prec;
    finalize(p->p);
    apply_tune_cache(p->p);
  } catch (...) {
    delete p;
    throw;
  }
  *plan = p;
  *C_meta = wrap_tensor(std::move(C));
  BST_CATCH
}

bst_status bst_permute_plan_c128(const bst_tensor* in, const char* const* new_order, bst_tensor** out_meta,
                                 bst_plan** plan) {
  BST_TRY
  if (!in || !out_meta || !plan || !new_order) fail(BST_E_INVALID, "null argument");
  *out_meta = nullptr;
  *plan = nullptr;
  const TensorDesc& T = *desc_of(in);
  std::vector<int> perm;
  for (int i = 0; i < T.rank(); ++i) {
    if (!new_order[i]) fail(BST_E_LABEL, "null label");
    const int k = T.label_index(new_order[i]);
    if (k < 0) fail(BST_E_LABEL, std::string("unknown label '") + new_order[i] + "'");
    if (std::find(perm.begin(), perm.end(), k) != perm.end())
      fail(BST_E_LABEL, std::string("label listed twice '") + new_order[i] + "'");
    perm.push_back(k);
  }
  std::unique_ptr<TensorDesc> out;
  auto* p = new_plan();
  try {
    permute_c128_plan(T, perm, p->p, out);
    finalize(p->p);
  } catch (...) {
    delete p;
    throw;
  }
  *plan = p;
  *out_meta = wrap_tensor(std::move(out));
  BST_CATCH
}

bst_status bst_contract_plan_c128(const bst_tensor* A, const bst_tensor* B, bst_precision prec,
                                  bst_tensor** C_meta, bst_plan** plan) {
  BST_TRY
  if (!A || !B || !C_meta || !plan) fail(BST_E_INVALID, "null argument");
  *C_meta = nullptr;
  *plan = nullptr;
  if (prec < BST_FP64 || prec > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  std::unique_ptr<TensorDesc> C;
  auto* p = new_plan();
  try {
    contract_c128_plan(*desc_of(A), *desc_of(B), p->p, C);
    p->p.prec = prec;
    finalize(p->p);
    apply_tune_cache(p->p);
  } catch (...) {
    delete p;
    throw;
  }
  *plan = p;
  *C_meta = wrap_tensor(std::move(C));
  BST_CATCH
}

bst_status bst_heff_plan(const bst_tensor* L, const bst_tensor* W1, const bst_tensor* W2,
                         const bst_tensor* R, const bst_tensor* psi, bst_precision prec,
                         bst_plan** plan) {
  BST_TRY
  if (!L || !W1 || !W2 || !R || !psi || !plan) fail(BST_E_INVALID, "null argument");
  *plan = nullptr;
  if (prec < BST_FP64 || prec > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  auto* p = new_plan();
  try {
    heff_plan(*desc_of(L), *desc_of(W1), *desc_of(W2), *desc_of(R), *desc_of(psi), p->p);
    p->p.prec = prec;
    finalize(p->p);
    apply_tune_cache(p->p);
  } catch (...) {
    delete p;
    throw;
  }
  *plan = p;
  BST_CATCH
}

bst_status bst_heff_batch_plan(int32_t n, const bst_plan* const* plans, bst_plan** batch) {
  BST_TRY
  if (n < 1 || !plans || !batch) fail(BST_E_INVALID, "bad batch arguments");
  *batch = nullptr;
  std::vector<const PlanData*> subs;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) fail(BST_E_INVALID, "null plan");
    subs.push_back(&plans[i]->p);
  }
  auto* p = new_plan();
  try {
    heff_batch(subs, p->p);
    p->p.prec = subs[0]->prec;
    finalize(p->p);
    apply_tune_cache(p->p);
  } catch (...) {
    delete p;
    throw;
  }
  *batch = p;
  BST_CATCH
}

bst_status bst_plan_workspace(const bst_plan* p, size_t* bytes) {
  BST_TRY
  if (!p || !bytes) fail(BST_E_INVALID, "null argument");
  *bytes = p->p.ws_bytes;
  BST_CATCH
}

bst_status bst_plan_info(const bst_plan* p, bst_plan_stats* st) {
  BST_TRY
  if (!p || !st) fail(BST_E_INVALID, "null argument");
  std::memset(st, 0, sizeof(*st));
  const PlanData& P = p->p;
  for (const auto& s : P.steps) {
    st->flops += s.flops;
    st->bytes += s.bytes;
    if (s.kind == StepKind::Gemm) {
      st->gemm_flops += s.flops;
      st->gemm_problems += (int64_t)s.probs.size();
      const int t = default_tile(s, P.prec);
      const auto& sh = gemm_tile_shapes(P.prec)[t];
      auto it = s.tile_lists.find({sh.bm, sh.bn});
      if (it != s.tile_lists.end()) st->gemm_tiles += it->second.second;
    }
  }
  st->launches = (int64_t)P.steps.size();
  st->nsteps = (int32_t)P.steps.size();
  BST_CATCH
}

bst_status bst_plan_step_info(const bst_plan* p, int32_t step, bst_step_info* info) {
  BST_TRY
  if (!p || !info) fail(BST_E_INVALID, "null argument");
  const PlanData& P = p->p;
  if (step < 0 || step >= (int32_t)P.steps.size()) fail(BST_E_INVALID, "step out of range");
  const Step& s = P.steps[step];
  std::memset(info, 0, sizeof(*info));
  std::strncpy(info->name, s.name.c_str(), sizeof(info->name) - 1);
  info->flops = s.flops;
  info->bytes_fp64 = s.bytes;
  info->bytes_fp32 = s.bytes32;
  if (s.kind == StepKind::Gemm) {
    const int t = default_tile(s, P.prec);
    const auto& sh = gemm_tile_shapes(P.prec)[t];
    auto it = s.tile_lists.find({sh.bm, sh.bn});
    info->items = it == s.tile_lists.end() ? 0 : it->second.second;
  } else {
    info->items = s.n0;
  }
  BST_CATCH
}

bst_status bst_plan_set_precision(bst_plan* p, bst_precision prec) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  if (prec < BST_FP64 || prec > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  p->p.prec = prec;
  BST_CATCH
}

bst_status bst_plan_tiles(const bst_plan* p, char* buf, size_t cap) {
  BST_TRY
  if (!p || !buf || cap == 0) fail(BST_E_INVALID, "null argument");
  std::string s;
  const PlanData& P = p->p;
  for (const auto& st : P.steps) {
    if (st.kind == StepKind::HApply) {
      if (st.fused.ok && fused_active(P, P.prec)) {
        s += st.name + ":fused64x64;";   // L.psi formed inside the MPO step
        continue;
      }
      const bool o32 = uses_planes(P, P.prec) && st.has_alt ? st.mpo_off32_alt : st.mpo_off32;
      s += st.name + (o32 ? ":i32;" : ":i64;");
      continue;
    }
    if (st.kind != StepKind::Gemm) continue;
    if (st.fusable && fused_active(P, P.prec)) continue;
    const bool pl = uses_planes(P, P.prec) && st.has_alt;
    const TileShape sh = pl ? gemm_planes_shapes(plane_count(P.prec))[planes_tile(st, P.prec)]
                            : gemm_tile_shapes(P.prec)[default_tile(st, P.prec)];
    const std::string kind = sh.direct == 1   ? "d"
                             : sh.direct == 3 ? "s" + std::to_string(sh.stages) + "w" + std::to_string(sh.waves)
                                              : "l";
    s += st.name + ":" + std::to_string(sh.bm) + "x" + std::to_string(sh.bn) + kind + (pl ? "p" : "") + ";";
  }
  std::strncpy(buf, s.c_str(), cap - 1);
  buf[cap - 1] = 0;
  BST_CATCH
}

}  // extern "C"

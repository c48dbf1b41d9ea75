// Symmetric SVD with truncation (Sec. "Singular value decomposition"):
// host bookkeeping.  The plan groups the blocks of a tensor seen as a matrix
// (first rowrank legs = rows) into one block matrix per charge of the new
// bond, lays the sector matrices, their rotation accumulators and singular
// values out in the caller's workspace and uploads the gather and sector
// tables; execute runs the SVD of every sector on the device; truncate picks
// the kept values across sectors on the device and returns their counts;
// factors / write produce the truncated U, singular values and V^dagger in
// the canonical block layout.
//
// New-bond sector order: as the charges first appear when the column-leg
// sector tuples are enumerated lexicographically (for one outgoing column
// leg, that leg's order).  Rows and columns of a sector matrix: the row
// (column) tuples in lexicographic order, each tuple's elements row-major.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>

#include "plan.h"
#include "svd.h"

namespace bst {

namespace {
struct Tuple {
  std::vector<int32_t> t;   // sector index per leg of the group
  int64_t start, ext;       // first row (column) in the sector matrix, extent
};
struct Sector {
  std::vector<int32_t> charge;   // one component per symmetry
  std::vector<Tuple> rows, cols;
  int64_t m = 0, n = 0;
  SvdSec dev{};
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

struct SvdPlanData {
  std::unique_ptr<TensorDesc> in;
  int rowrank = 0;
  int nsym = 1;
  std::vector<int32_t> moduli;
  std::vector<Sector> secs;
  int64_t nvalues = 0;
  // workspace layout (bytes)
  size_t ws_tab = 0, ws_secs = 0, ws_gjobs = 0, ws_gwork = 0, ws_x = 0, ws_v = 0, ws_sig = 0, ws_sorted = 0,
         ws_perm = 0, ws_sweeps = 0, ws_kept = 0, ws_serr = 0, ws_mb = 0, ws_wtab = 0, ws_bytes = 0;
  size_t wtab_cap = 0;   // bytes reserved for the write tables
  // sectors rotated a round per launch (X larger than the LDS budget)
  std::vector<int32_t> big;
  size_t ws_big = 0, ws_flags = 0;
  int32_t rounds = 0, pairs = 0;
  int64_t vmax = 0;
  std::vector<uint8_t> blob;   // sector and gather tables
  int64_t ngwork = 0;
  void* uploaded = nullptr;
  // a second stream (default priority) on which the sectors that fit LDS
  // run their sweeps beside the big sectors' rounds; made on first use, on
  // the device then current
  hipStream_t aux = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int aux_dev = -1;
  void release_aux() {
    if (!aux) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(aux_dev);
    (void)hipStreamDestroy(aux);
    for (auto& e : ev) (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
    aux = nullptr;
    ev[0] = ev[1] = nullptr;
    aux_dev = -1;
  }
  ~SvdPlanData() { release_aux(); }
};

}  // namespace bst

struct bst_svd {
  bst::SvdPlanData p;
};

namespace bst {

namespace {
// Combined flux of legs [l0, l1) for a tuple of their sector indices.
std::vector<int32_t> group_flux(const TensorDesc& T, int l0, int l1, const std::vector<int32_t>& t) {
  const int ns = T.legs[l0].nsym();
  std::vector<int32_t> f(ns, 0);
  for (int c = 0; c < ns; ++c) {
    int64_t s = 0;
    for (int l = l0; l < l1; ++l) s += (int64_t)T.legs[l].dir * T.legs[l].charge(t[l - l0], c);
    const int32_t n = T.legs[l0].modulus(c);
    f[c] = (int32_t)(n >= 2 ? ((s % n) + n) % n : s);
  }
  return f;
}

std::vector<int32_t> negate(const std::vector<int32_t>& q, const std::vector<int32_t>& moduli) {
  std::vector<int32_t> r(q.size());
  for (size_t c = 0; c < q.size(); ++c) {
    const int32_t n = c < moduli.size() ? moduli[c] : 0;
    r[c] = n >= 2 ? (int32_t)(((-(int64_t)q[c]) % n + n) % n) : -q[c];
  }
  return r;
}

// All sector tuples of legs [l0, l1), lexicographic (first leg slowest).
std::vector<std::vector<int32_t>> tuples(const TensorDesc& T, int l0, int l1) {
  std::vector<std::vector<int32_t>> out;
  std::vector<int32_t> t(l1 - l0, 0);
  if (l1 <= l0) return out;
  while (true) {
    out.push_back(t);
    int i = l1 - l0 - 1;
    while (i >= 0) {
      if (++t[i] < (int32_t)T.legs[l0 + i].q.size()) break;
      t[i] = 0;
      --i;
    }
    if (i < 0) break;
    if (out.size() > ((size_t)1 << 24)) fail(BST_E_INVALID, "too many sector tuples");
  }
  return out;
}

int64_t extent(const TensorDesc& T, int l0, const std::vector<int32_t>& t) {
  int64_t e = 1;
  for (size_t i = 0; i < t.size(); ++i) e *= T.legs[l0 + i].g[t[i]];
  return e;
}

template <typename V>
size_t put(std::vector<uint8_t>& blob, const std::vector<V>& v) {
  const size_t off = align256(blob.size());
  blob.resize(off + std::max<size_t>(v.size() * sizeof(V), 1));
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(V));
  return off;
}

void build(SvdPlanData& P) {
  const TensorDesc& T = *P.in;
  const int r = P.rowrank, rank = T.rank();
  P.nsym = T.legs[0].nsym();
  P.moduli = T.legs[0].sym;
  const auto rt = tuples(T, 0, r), ct = tuples(T, r, rank);
  // sectors in order of first appearance over the column tuples
  std::map<std::vector<int32_t>, int> index;
  for (const auto& c : ct) {
    const auto q = negate(group_flux(T, r, rank, c), P.moduli);
    if (index.count(q)) continue;
    index[q] = (int)P.secs.size();
    Sector s;
    s.charge = q;
    P.secs.push_back(std::move(s));
  }
  for (const auto& t : rt) {
    auto it = index.find(group_flux(T, 0, r, t));
    if (it == index.end()) continue;
    Sector& s = P.secs[it->second];
    const int64_t e = extent(T, 0, t);
    s.rows.push_back({t, s.m, e});
    s.m += e;
  }
  for (const auto& t : ct) {
    Sector& s = P.secs[index.at(negate(group_flux(T, r, rank, t), P.moduli))];
    const int64_t e = extent(T, r, t);
    s.cols.push_back({t, s.n, e});
    s.n += e;
  }
  // drop sectors with no rows (no block of T reaches them)
  std::vector<Sector> kept;
  for (auto& s : P.secs)
    if (s.m > 0 && s.n > 0) kept.push_back(std::move(s));
  P.secs = std::move(kept);
  // device layout of the sector matrices
  int64_t xo = 0, vo = 0, so = 0;
  std::vector<SvdSec> dsecs;
  for (auto& s : P.secs) {
    if (s.m > 0x7FFFFFFF || s.n > 0x7FFFFFFF) fail(BST_E_INVALID, "sector matrix too large");
    const int64_t rr = std::min(s.m, s.n);
    s.dev.x_off = xo;
    s.dev.v_off = vo;
    s.dev.s_off = so;
    s.dev.m = (int32_t)s.m;
    s.dev.n = (int32_t)s.n;
    xo += s.m * s.n;
    vo += rr * rr;
    so += rr;
    dsecs.push_back(s.dev);
  }
  P.nvalues = so;
  if (so > 0x7FFFFFFF) fail(BST_E_INVALID, "too many singular values");
  P.big.clear();
  P.rounds = P.pairs = 0;
  P.vmax = 0;
  for (size_t k = 0; k < P.secs.size(); ++k) {
    const int64_t m = P.secs[k].m, n = P.secs[k].n;
    if (!svd_sector_is_big(m, n)) continue;
    const int64_t r = std::min(m, n), rr = r + (r & 1);
    P.big.push_back((int32_t)k);
    P.rounds = (int32_t)std::max<int64_t>(P.rounds, rr - 1);
    P.pairs = (int32_t)std::max<int64_t>(P.pairs, rr / 2);
    P.vmax = std::max(P.vmax, r * r);
  }
  if (P.big.size() > 65535) fail(BST_E_INVALID, "more than 65535 sector matrices above the LDS budget");
  // gather jobs: every block of T into its sector matrix
  std::vector<SvdGather> gj;
  std::vector<SvdWork> gw;
  std::map<std::vector<int32_t>, std::pair<int, int64_t>> rpos, cpos;   // tuple -> (sector, start)
  for (size_t k = 0; k < P.secs.size(); ++k) {
    for (const auto& t : P.secs[k].rows) rpos[t.t] = {(int)k, t.start};
    for (const auto& t : P.secs[k].cols) cpos[t.t] = {(int)k, t.start};
  }
  for (int64_t b = 0; b < T.nblocks; ++b) {
    const int32_t* qn = T.block_qn(b);
    std::vector<int32_t> rt1(qn, qn + r), ct1(qn + r, qn + rank);
    const auto ri = rpos.find(rt1);
    const auto ci = cpos.find(ct1);
    if (ri == rpos.end() || ci == cpos.end() || ri->second.first != ci->second.first)
      fail(BST_E_INVALID, "internal: block outside the sector matrices");
    const Sector& s = P.secs[ri->second.first];
    SvdGather g{};
    g.in_off = T.offset[b];
    g.x_off = s.dev.x_off;
    g.rows = (int32_t)extent(T, 0, rt1);
    g.cols = (int32_t)extent(T, r, ct1);
    g.row0 = (int32_t)ri->second.second;
    g.col0 = (int32_t)ci->second.second;
    g.m = s.dev.m;
    g.n = s.dev.n;
    const int32_t jid = (int32_t)gj.size();
    gj.push_back(g);
    const int64_t total = (int64_t)g.rows * g.cols;
    for (int64_t st = 0; st < total; st += kSvdGatherChunk) gw.push_back({jid, (int32_t)st});
  }
  P.ngwork = (int64_t)gw.size();
  P.blob.clear();
  P.ws_secs = put(P.blob, dsecs);
  P.ws_gjobs = put(P.blob, gj);
  P.ws_gwork = put(P.blob, gw);
  P.ws_big = put(P.blob, P.big);
  size_t off = align256(P.blob.size());
  P.ws_tab = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 8));
    return o;
  };
  P.ws_x = take(sizeof(double) * (size_t)xo);
  P.ws_v = take(sizeof(double) * (size_t)vo);
  P.ws_sig = take(sizeof(double) * (size_t)so);
  P.ws_sorted = take(sizeof(double) * (size_t)so);
  P.ws_perm = take(sizeof(int32_t) * (size_t)so);
  P.ws_sweeps = take(sizeof(int32_t) * P.secs.size());
  P.ws_kept = take(sizeof(int64_t) * P.secs.size());
  P.ws_serr = take(sizeof(double));
  P.ws_mb = take(sizeof(int64_t) * P.secs.size());
  P.ws_flags = take(sizeof(int32_t) * 2 * P.big.size());
  // write tables: one job per block of U and V^dagger and one per S sector,
  // work items of kSvdGatherChunk elements
  int64_t wjobs = 2 * (int64_t)P.secs.size();
  int64_t wwork = 2 * (int64_t)P.secs.size();
  for (const auto& s : P.secs) {
    wjobs += (int64_t)s.rows.size() + (int64_t)s.cols.size();
    const int64_t k = std::min(s.m, s.n);
    for (const auto& t : s.rows) wwork += (t.ext * k + kSvdGatherChunk - 1) / kSvdGatherChunk;
    for (const auto& t : s.cols) wwork += (t.ext * k + kSvdGatherChunk - 1) / kSvdGatherChunk;
  }
  P.wtab_cap = align256(sizeof(SvdWrite) * (size_t)wjobs) + align256(sizeof(SvdWriteWork) * (size_t)wwork) + 256;
  P.ws_wtab = take(P.wtab_cap);
  P.ws_bytes = off;
}

void upload(SvdPlanData& P, void* ws, hipStream_t s) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) fail(BST_E_INVALID, "workspace must be non-null and 256-byte aligned");
  if (P.uploaded == ws) return;
  check_hip(hipMemcpyAsync(ws, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice, s), "svd tables");
  check_hip(hipStreamSynchronize(s), "svd tables");
  P.uploaded = ws;
}

template <typename V>
V* at(void* ws, size_t off) {
  return reinterpret_cast<V*>(static_cast<char*>(ws) + off);
}

// Output descriptors of the kept sectors: U[rows..., bond] and V^dagger[bond, cols...].
void factor_legs(const SvdPlanData& P, const int64_t* kept, const std::string& bond, std::vector<LegDesc>& ul,
                 std::vector<LegDesc>& vl) {
  const TensorDesc& T = *P.in;
  LegDesc b;
  b.sym = P.moduli;
  b.label = bond;
  for (size_t k = 0; k < P.secs.size(); ++k) {
    if (kept[k] < 0 || kept[k] > std::min(P.secs[k].m, P.secs[k].n))
      fail(BST_E_INVALID, "kept count outside 0..min(rows, cols) of its sector");
    if (kept[k] == 0) continue;
    b.q.push_back(P.secs[k].charge[0]);
    for (int c = 1; c < P.nsym; ++c) b.qx.push_back(P.secs[k].charge[c]);
    b.g.push_back(kept[k]);
  }
  if (b.q.empty()) fail(BST_E_INVALID, "every sector truncated away");
  ul.assign(T.legs.begin(), T.legs.begin() + P.rowrank);
  vl.assign(T.legs.begin() + P.rowrank, T.legs.end());
  for (const auto& l : ul)
    if (l.label == bond) fail(BST_E_LABEL, "bond label equals a row leg label");
  for (const auto& l : vl)
    if (l.label == bond) fail(BST_E_LABEL, "bond label equals a column leg label");
  b.dir = -1;
  ul.push_back(b);
  b.dir = 1;
  vl.insert(vl.begin(), b);
}
}  // namespace

}  // namespace bst

using namespace bst;

extern "C" {

bst_status bst_svd_plan(const bst_tensor* M, int32_t rowrank, bst_svd** out) {
  BST_TRY
  if (!M || !out) fail(BST_E_INVALID, "null argument");
  *out = nullptr;
  const TensorDesc& T = *M->d;
  if (rowrank < 1 || rowrank >= T.rank()) fail(BST_E_INVALID, "rowrank must leave >= 1 row and >= 1 column leg");
  auto p = std::make_unique<bst_svd>();
  p->p.in = std::make_unique<TensorDesc>(T);
  p->p.rowrank = rowrank;
  build(p->p);
  *out = p.release();
  BST_CATCH
}

bst_status bst_svd_info(const bst_svd* p, int32_t* nsectors, int64_t* nvalues, size_t* ws_bytes) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  if (nsectors) *nsectors = (int32_t)p->p.secs.size();
  if (nvalues) *nvalues = p->p.nvalues;
  if (ws_bytes) *ws_bytes = p->p.ws_bytes;
  BST_CATCH
}

bst_status bst_svd_sector(const bst_svd* p, int32_t k, int32_t* charge, int64_t* rows, int64_t* cols) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  if (k < 0 || k >= (int32_t)p->p.secs.size()) fail(BST_E_INVALID, "sector index out of range");
  const auto& s = p->p.secs[k];
  if (charge)
    for (int c = 0; c < p->p.nsym; ++c) charge[c] = s.charge[c];
  if (rows) *rows = s.m;
  if (cols) *cols = s.n;
  BST_CATCH
}

bst_status bst_svd_execute(bst_svd* p, const void* M, void* ws, void* stream) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  SvdPlanData& P = p->p;
  if (!M && P.in->numel > 0) fail(BST_E_INVALID, "null input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  check_hip(hipGetLastError(), "pending device error");
  upload(P, ws, s);
  SvdLaunch l{};
  l.gjobs = at<const SvdGather>(ws, P.ws_gjobs);
  l.gwork = at<const SvdWork>(ws, P.ws_gwork);
  l.ngwork = P.ngwork;
  l.secs = at<const SvdSec>(ws, P.ws_secs);
  l.nsec = (int32_t)P.secs.size();
  l.in = static_cast<const double*>(M);
  l.X = at<double>(ws, P.ws_x);
  l.V = at<double>(ws, P.ws_v);
  l.sig = at<double>(ws, P.ws_sig);
  l.sorted = at<double>(ws, P.ws_sorted);
  l.perm = at<int32_t>(ws, P.ws_perm);
  l.sweeps = at<int32_t>(ws, P.ws_sweeps);
  l.big = at<const int32_t>(ws, P.ws_big);
  l.nbig = (int32_t)P.big.size();
  l.rounds = P.rounds;
  l.pairs = P.pairs;
  l.vmax = P.vmax;
  l.flags = at<int32_t>(ws, P.ws_flags);
  check_hip(launch_svd_gather(l, s), "svd gather");
  if (l.nbig == 0) {
    check_hip(launch_svd_finish(l, s, 0), "svd");
  } else {
    // the sectors that fit run their sweeps on the second stream meanwhile
    int dev = -1;
    check_hip(hipGetDevice(&dev), "device");
    if (P.aux && P.aux_dev != dev) P.release_aux();
    if (!P.aux) {
      check_hip(hipStreamCreateWithFlags(&P.aux, hipStreamNonBlocking), "svd stream");
      P.aux_dev = dev;
      for (auto& e : P.ev) check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "svd event");
    }
    check_hip(hipEventRecord(P.ev[0], s), "svd event");
    check_hip(hipStreamWaitEvent(P.aux, P.ev[0], 0), "svd event");
    check_hip(launch_svd_finish(l, P.aux, 1), "svd");
    check_hip(hipEventRecord(P.ev[1], P.aux), "svd event");
    {
      // sweeps of the big sectors until each has had one without a rotation
      // (at most kSvdMaxSweeps): the host reads the flags after every sweep
      std::vector<int32_t> fl(2 * (size_t)l.nbig);
      for (int sw = 0; sw < kSvdMaxSweeps; ++sw) {
        check_hip(launch_svd_sweep(l, s), "svd sweep");
        check_hip(hipMemcpyAsync(fl.data(), l.flags, sizeof(int32_t) * fl.size(), hipMemcpyDeviceToHost, s),
                  "svd flags");
        check_hip(hipStreamSynchronize(s), "svd flags");
        bool all = true;
        for (int b = 0; b < l.nbig; ++b) all = all && fl[2 * (size_t)b + 1] != 0;
        if (all) break;
      }
    }
    check_hip(hipStreamWaitEvent(s, P.ev[1], 0), "svd event");
    check_hip(launch_svd_finish(l, s, 2), "svd");
  }
  BST_CATCH
}

bst_status bst_svd_truncate(bst_svd* p, int64_t keepdim, double err, const int64_t* min_blockdim, void* ws,
                            void* stream, int64_t* kept, double* s_err) {
  BST_TRY
  if (!p || !kept) fail(BST_E_INVALID, "null argument");
  SvdPlanData& P = p->p;
  if (keepdim < 0) fail(BST_E_INVALID, "keepdim must be >= 0");
  if (!(err >= 0.0)) fail(BST_E_INVALID, "err must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  upload(P, ws, s);
  const int ns = (int)P.secs.size();
  if (min_blockdim) {
    for (int k = 0; k < ns; ++k)
      if (min_blockdim[k] < 0) fail(BST_E_INVALID, "min_blockdim entries must be >= 0");
    check_hip(hipMemcpyAsync(at<int64_t>(ws, P.ws_mb), min_blockdim, sizeof(int64_t) * (size_t)ns,
                             hipMemcpyHostToDevice, s),
              "min_blockdim");
  }
  SvdSelectLaunch l{};
  l.secs = at<const SvdSec>(ws, P.ws_secs);
  l.nsec = ns;
  l.sorted = at<const double>(ws, P.ws_sorted);
  l.min_blockdim = min_blockdim ? at<const int64_t>(ws, P.ws_mb) : nullptr;
  l.keepdim = keepdim;
  l.err = err;
  l.kept = at<int64_t>(ws, P.ws_kept);
  l.s_err = at<double>(ws, P.ws_serr);
  if (ns > 0) check_hip(launch_svd_select(l, s), "svd truncation");
  std::vector<int64_t> hk((size_t)ns);
  double he = 0.0;
  if (ns > 0) {
    check_hip(hipMemcpyAsync(hk.data(), l.kept, sizeof(int64_t) * (size_t)ns, hipMemcpyDeviceToHost, s), "kept");
    check_hip(hipMemcpyAsync(&he, l.s_err, sizeof(double), hipMemcpyDeviceToHost, s), "s_err");
  }
  check_hip(hipStreamSynchronize(s), "svd truncation");
  for (int k = 0; k < ns; ++k) kept[k] = hk[k];
  if (s_err) *s_err = he;
  BST_CATCH
}

bst_status bst_svd_factors(const bst_svd* p, const int64_t* kept, const char* bond, bst_tensor** U,
                           bst_tensor** Vd) {
  BST_TRY
  if (!p || !kept || !bond || !U || !Vd) fail(BST_E_INVALID, "null argument");
  *U = *Vd = nullptr;
  std::vector<LegDesc> ul, vl;
  factor_legs(p->p, kept, bond, ul, vl);
  auto u = wrap_tensor(make_tensor(std::move(ul)));
  try {
    *Vd = wrap_tensor(make_tensor(std::move(vl)));
  } catch (...) {
    delete u;
    throw;
  }
  *U = u;
  BST_CATCH
}

bst_status bst_svd_write(bst_svd* p, const int64_t* kept, int32_t absorb, void* U, void* S, void* Vd, void* ws,
                         void* stream) {
  BST_TRY
  if (!p || !kept) fail(BST_E_INVALID, "null argument");
  if (absorb < 0 || absorb > 2) fail(BST_E_INVALID, "absorb must be 0, 1 (into U) or 2 (into V^dagger)");
  SvdPlanData& P = p->p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  upload(P, ws, s);
  std::vector<LegDesc> ul, vl;
  factor_legs(P, kept, "_bond_", ul, vl);
  const auto Ut = make_tensor(std::move(ul));
  const auto Vt = make_tensor(std::move(vl));
  if ((!U && Ut->numel) || (!Vd && Vt->numel) || !S) fail(BST_E_INVALID, "null output");
  const int r = P.rowrank, rank = P.in->rank();
  std::vector<SvdWrite> jobs;
  std::vector<SvdWriteWork> work;
  auto add = [&](const SvdWrite& j, int64_t total) {
    const int32_t id = (int32_t)jobs.size();
    jobs.push_back(j);
    for (int64_t st = 0; st < total; st += kSvdGatherChunk) work.push_back({id, (int32_t)st});
  };
  int pos = 0;
  int64_t soff = 0;
  std::vector<int32_t> key(rank + 1);
  for (size_t k = 0; k < P.secs.size(); ++k) {
    const Sector& sec = P.secs[k];
    const int64_t kk = kept[k];
    if (kk == 0) continue;
    for (const auto& t : sec.rows) {
      for (int i = 0; i < r; ++i) key[i] = t.t[i];
      key[r] = pos;
      const int64_t b = Ut->find(key.data());
      if (b < 0) fail(BST_E_INVALID, "internal: U block missing");
      add({Ut->offset[b], (int32_t)k, 0, (int32_t)t.start, (int32_t)t.ext, (int32_t)kk, 0}, t.ext * kk);
    }
    for (const auto& t : sec.cols) {
      key[0] = pos;
      for (int i = 0; i < rank - r; ++i) key[1 + i] = t.t[i];
      const int64_t b = Vt->find(key.data());
      if (b < 0) fail(BST_E_INVALID, "internal: V^dagger block missing");
      add({Vt->offset[b], (int32_t)k, 1, (int32_t)t.start, (int32_t)t.ext, (int32_t)kk, 0}, t.ext * kk);
    }
    add({soff, (int32_t)k, 2, 0, (int32_t)kk, (int32_t)kk, 0}, kk);
    soff += kk;
    ++pos;
  }
  std::vector<uint8_t> tab;
  const size_t jo = put(tab, jobs), wo = put(tab, work);
  if (tab.size() > P.wtab_cap) fail(BST_E_INVALID, "internal: write tables exceed their reserve");
  check_hip(hipMemcpyAsync(at<uint8_t>(ws, P.ws_wtab), tab.data(), tab.size(), hipMemcpyHostToDevice, s),
            "svd write tables");
  SvdWriteLaunch l{};
  l.jobs = at<const SvdWrite>(ws, P.ws_wtab + jo);
  l.work = at<const SvdWriteWork>(ws, P.ws_wtab + wo);
  l.nwork = (int64_t)work.size();
  l.secs = at<const SvdSec>(ws, P.ws_secs);
  l.X = at<const double>(ws, P.ws_x);
  l.V = at<const double>(ws, P.ws_v);
  l.sorted = at<const double>(ws, P.ws_sorted);
  l.perm = at<const int32_t>(ws, P.ws_perm);
  l.absorb = absorb;
  l.U = static_cast<double*>(U);
  l.Vd = static_cast<double*>(Vd);
  l.S = static_cast<double*>(S);
  check_hip(launch_svd_write(l, s), "svd write");
  // the host copy of the tables must outlive the transfer
  check_hip(hipStreamSynchronize(s), "svd write");
  BST_CATCH
}

bst_status bst_svd_sweeps(const bst_svd* p, const void* ws, void* stream, int32_t* sweeps) {
  BST_TRY
  if (!p || !ws || !sweeps) fail(BST_E_INVALID, "null argument");
  const SvdPlanData& P = p->p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!P.secs.empty()) {
    check_hip(hipMemcpyAsync(sweeps, static_cast<const char*>(ws) + P.ws_sweeps, sizeof(int32_t) * P.secs.size(),
                             hipMemcpyDeviceToHost, s),
              "svd sweeps");
    check_hip(hipStreamSynchronize(s), "svd sweeps");
  }
  BST_CATCH
}

bst_status bst_svd_forget_workspace(bst_svd* p) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  p->p.uploaded = nullptr;
  BST_CATCH
}

bst_status bst_svd_destroy(bst_svd* p) {
  delete p;
  set_last_error("");
  return BST_OK;
}

}  // extern "C"

// Plan execution: workspace layout, device pointer tables, hipGraph replay,
// per-step timing and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

#include "plan.h"

namespace bst {

// Which plan's tables a workspace currently holds.
static std::mutex g_ws_mu;
static std::map<void*, uint64_t> g_ws_owner;

hipError_t launch_set_ptrs(void** table, void* const* src, int n, hipStream_t s);

std::vector<void*> build_ptrs(PlanData& P, const void* const* in, void* const* out, void* ws) {
  std::vector<void*> ptrs((size_t)std::max(P.nslots, 1), nullptr);
  for (size_t k = 0; k < P.in_slots.size(); ++k) {
    const bool empty = k < P.in_numel.size() && P.in_numel[k] == 0;
    if ((!in || !in[k]) && !empty) fail(BST_E_INVALID, "null input pointer " + std::to_string(k));
    ptrs[P.in_slots[k]] = in ? const_cast<void*>(in[k]) : nullptr;
  }
  for (size_t k = 0; k < P.out_slots.size(); ++k) {
    const bool empty = k < P.out_numel.size() && P.out_numel[k] == 0;
    if ((!out || !out[k]) && !empty) fail(BST_E_INVALID, "null output pointer " + std::to_string(k));
    ptrs[P.out_slots[k]] = out ? out[k] : nullptr;
  }
  for (const auto& ib : P.internals) ptrs[ib.slot] = static_cast<char*>(ws) + ib.ws_off;
  return ptrs;
}

void* upload_table(PlanData& P, const std::vector<void*>& ptrs, void* ws, size_t off,
                   hipStream_t s) {
  (void)P;
  void** table = reinterpret_cast<void**>(static_cast<char*>(ws) + off);
  check_hip(launch_set_ptrs(table, ptrs.data(), (int)ptrs.size(), s), "pointer table");
  return table;
}

void* prepare_ws(PlanData& P, const void* const* in, void* const* out, void* ws, hipStream_t s) {
  if (!ws) fail(BST_E_INVALID, "null workspace");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) fail(BST_E_INVALID, "workspace must be 256-byte aligned");
  auto ptrs = build_ptrs(P, in, out, ws);
  bool need_blob;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws_owner.find(ws);
    need_blob = (it == g_ws_owner.end() || it->second != P.id || P.uploaded_ws != ws);
  }
  if (need_blob) {
    if (!P.blob.empty()) {
      check_hip(hipMemcpyAsync(static_cast<char*>(ws) + P.ws_blob_off, P.blob.data(), P.blob.size(),
                               hipMemcpyHostToDevice, s),
                "plan table upload");
      check_hip(hipStreamSynchronize(s), "plan table upload");
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_ws_owner[ws] = P.id;
    P.uploaded_ws = ws;
    P.last_ptrs.clear();
  }
  if (ptrs != P.last_ptrs) {
    upload_table(P, ptrs, ws, P.ws_ptr_off, s);
    P.last_ptrs = ptrs;
  }
  return static_cast<char*>(ws) + P.ws_ptr_off;
}

bool uses_planes(const PlanData& P, bst_precision prec) {
  if (!P.has_planes) return false;
  if (prec == BST_BF16X3 || prec == BST_BF16X6) return true;
  if (prec != BST_FP64 || !P.f64_panels || std::getenv("BST_FP64_BLOCKS")) return false;
  return P.fp64_panels_on || std::getenv("BST_FP64_PANELS") != nullptr;
}

int plane_count(bst_precision prec) { return prec == BST_FP64 ? 1 : prec == BST_BF16X6 ? 3 : 2; }
int plane_count_of_key(int key) { return plane_count((bst_precision)(key - 10)); }

// The fused L.psi + MPO kernel runs for the two-plane forms when the plan
// has its schedule and the autotuner chose it; BST_FUSED_MPO=0 / 1
// overrides the choice.
bool fused_active(const PlanData& P, bst_precision prec) {
  if (!P.fused_ok || !uses_planes(P, prec) || plane_count(prec) != 2) return false;
  if (const char* e = std::getenv("BST_FUSED_MPO")) return std::strcmp(e, "0") != 0;
  return P.fused_on;
}

bool step_runs(const PlanData& P, const Step& st, bst_precision prec, bool skip_const) {
  if (skip_const && st.constant) return false;
  if (st.fusable && fused_active(P, prec)) return false;   // formed inside the fused MPO step
  if (st.kind == StepKind::Split && !uses_planes(P, prec)) return false;
  return true;
}

// Tile-choice key of the bfloat16-plane GEMM variant of a form.
static int planes_key(bst_precision prec) { return 10 + (int)prec; }

// LDS-staged 64x64: the fallback of the pipelined shapes (problems outside
// their layout rules)
constexpr int kPlanesDefaultTile = 0;

// Without a tuned choice: the largest pipelined tile, 128 x 256 for wide
// problems and 256 x 128 for tall ones (by the flop-weighted mean of M and
// N); the larger tile cuts the operand traffic from L2 more than its
// padding costs (measured on the H_eff GEMMs).  Falls back to a 128 x 128
// shape, then to the LDS-staged kernel.
static int planes_auto_tile(const Step& st, int np) {
  double wm = 0, wn = 0;
  for (const auto& p : st.probs_alt) {
    int64_t k = 0;
    for (int q = 0; q < p.seg_count; ++q) k += st.segs_alt[p.seg_begin + q].K;
    const double w = (double)p.M * (double)p.N * (double)std::max<int64_t>(k, 1);
    wm += w * p.M;
    wn += w * p.N;
  }
  const int want_bm = wn >= wm ? 128 : 256, want_bn = wn >= wm ? 256 : 128;
  const auto& shapes = gemm_planes_shapes(np);
  int best = kPlanesDefaultTile, rank = 0;
  for (size_t i = 0; i < shapes.size(); ++i) {
    const TileShape& sh = shapes[i];
    if (sh.direct != 3) continue;
    auto it = st.streams_alt.find(np * 64 + (int)i);
    if (it == st.streams_alt.end() || !it->second.ok) continue;
    const int r = (sh.bm == want_bm && sh.bn == want_bn) ? 2 : (sh.bm == 128 && sh.bn == 128) ? 1 : 0;
    if (r > rank) {
      rank = r;
      best = (int)i;
    }
  }
  return best;
}

int planes_tile(const Step& st, bst_precision prec) {
  auto it = st.tile_choice.find(planes_key(prec));
  if (it != st.tile_choice.end()) return it->second;
  return planes_auto_tile(st, plane_count(prec));
}

void run_steps_impl(PlanData& P, void* ws, void* const* dptrs, bst_precision prec, hipStream_t s,
                    bool skip_const, int only_step,
                    std::vector<std::pair<hipEvent_t, hipEvent_t>>* ev) {
  const char* blob = static_cast<const char*>(ws) + P.ws_blob_off;
  char* wsb = static_cast<char*>(ws);
  const ElemType inter = (prec == BST_FP64) ? ElemType::F64 : ElemType::F32;
  const bool planes = uses_planes(P, prec);
  const int np = plane_count(prec);
  for (size_t k = 0; k < P.steps.size(); ++k) {
    if (only_step >= 0 && (int)k != only_step) continue;
    Step& st = P.steps[k];
    if (!step_runs(P, st, prec, skip_const)) continue;
    if (ev) check_hip(hipEventRecord((*ev)[k].first, s), "event");
    hipError_t e = hipSuccess;
    switch (st.kind) {
      case StepKind::Split: {
        SplitLaunch l{};
        l.np = np;
        l.in_f32 = st.reads_psi && P.psi_f32;
        l.items = reinterpret_cast<const SplitItem*>(blob + st.off0);
        l.ptrs = dptrs;
        l.nwork = st.n0;
        e = launch_split(l, s);
        break;
      }
      case StepKind::Gemm: {
        if (planes && st.has_alt) {
          PlanesLaunch g{};
          g.np = np;
          g.tc = np == 1 ? ElemType::F64
                 : st.tc == Elem::Inter || (st.writes_out && P.z_f32) ? ElemType::F32 : ElemType::F64;
          g.tile = planes_tile(st, prec);
          if (gemm_planes_shapes(np)[g.tile].direct == 3) {
            auto sit = st.streams_alt.find(np * 64 + g.tile);
            if (sit != st.streams_alt.end() && sit->second.ok) {
              const auto& L = sit->second;
              StreamLaunch sl{};
              sl.np = np;
              sl.tc = g.tc;
              sl.tile = g.tile;
              sl.steps = reinterpret_cast<const KStep*>(blob + L.steps_off);
              sl.wg_begin = reinterpret_cast<const int64_t*>(blob + L.begin_off);
              sl.nwg = L.nwg;
              sl.ptrs = dptrs;
              sl.rowtab = reinterpret_cast<const int64_t*>(blob + L.rows_off);
              e = launch_gemm_planes_stream(sl, s);
              break;
            }
            if (np == 1) fail(BST_E_INVALID, "internal: float64 tile without a k-step schedule");
            g.tile = kPlanesDefaultTile;   // problems outside the kernel's layout rules
          }
          const auto& sh = gemm_planes_shapes(np)[g.tile];
          auto it = st.tile_lists_alt.find({sh.bm, sh.bn});
          if (it == st.tile_lists_alt.end()) fail(BST_E_INVALID, "internal: missing tile list");
          g.tiles = reinterpret_cast<const GemmTile*>(blob + it->second.first);
          g.ntiles = it->second.second;
          g.probs = reinterpret_cast<const GemmProb*>(blob + st.off3);
          g.segs = reinterpret_cast<const GemmSeg*>(blob + st.off2);
          g.rowmap = reinterpret_cast<const int64_t*>(blob + st.off5);
          g.ptrs = dptrs;
          e = launch_gemm_planes(g, s);
          break;
        }
        if (st.writes_out && P.z_f32) fail(BST_E_INVALID, "internal: float32 output needs the plane path");
        const bst_precision form = st.fixed_fp64 ? BST_FP64 : prec;
        GemmLaunch g{};
        g.form = form;
        g.ta = st.ta == Elem::Inter ? inter : ElemType::F64;
        g.tb = ElemType::F64;
        g.tc = st.tc == Elem::Inter ? inter : ElemType::F64;
        g.transb = st.transb;
        g.tile = default_tile(st, form);
        const auto& sh = gemm_tile_shapes(form)[g.tile];
        auto it = st.tile_lists.find({sh.bm, sh.bn});
        if (it == st.tile_lists.end()) fail(BST_E_INVALID, "internal: missing tile list");
        g.tiles = reinterpret_cast<const GemmTile*>(blob + it->second.first);
        g.ntiles = it->second.second;
        g.probs = reinterpret_cast<const GemmProb*>(blob + st.off0);
        g.segs = reinterpret_cast<const GemmSeg*>(blob + st.off1);
        g.ptrs = dptrs;
        e = launch_gemm(g, s);
        break;
      }
      case StepKind::Expand: {
        ExpandLaunch xl{reinterpret_cast<const ExpandJob*>(blob + st.off0),
                        reinterpret_cast<const ExpandWork*>(blob + st.off1), dptrs, st.n0};
        e = launch_expand(xl, s);
        break;
      }
      case StepKind::Permute: {
        PermLaunch pl{reinterpret_cast<const PermJob*>(blob + st.off0),
                      reinterpret_cast<const PermWork*>(blob + st.off1), dptrs, st.n0};
        e = launch_permute(pl, s);
        break;
      }
      case StepKind::HCoef: {
        HCoefLaunch c{};
        c.terms = reinterpret_cast<const HTerm*>(blob + st.off0);
        c.entry_begin = reinterpret_cast<const int32_t*>(blob + st.off1);
        c.nentries = st.n0;
        c.ptrs = dptrs;
        c.nmax = st.nmax;
        c.coef64 = reinterpret_cast<double*>(wsb + P.ws_coef64_off);
        c.coef32 = reinterpret_cast<float*>(wsb + P.ws_coef32_off);
        c.cnt = reinterpret_cast<int32_t*>(wsb + P.ws_cnt_off);
        c.idx = reinterpret_cast<int32_t*>(wsb + P.ws_idx_off);
        c.val64 = reinterpret_cast<double*>(wsb + P.ws_val64_off);
        c.val32 = reinterpret_cast<float*>(wsb + P.ws_val32_off);
        e = launch_hcoef(c, s);
        break;
      }
      case StepKind::HApply: {
        if (planes && st.has_alt && st.fused.ok && fused_active(P, prec)) {
          LhFusedLaunch f{};
          f.nmax = st.nmax;
          f.steps = reinterpret_cast<const KStep*>(blob + st.fused.steps_off);
          f.wg_begin = reinterpret_cast<const int64_t*>(blob + st.fused.begin_off);
          f.nwg = st.fused.nwg;
          f.ptrs = dptrs;
          f.coef = reinterpret_cast<const float*>(wsb + P.ws_coef32_off);
          f.planes = reinterpret_cast<const HPlane*>(blob + st.fused_planes_off);
          f.out_slot = st.tasks_alt.empty() ? 11 : st.tasks_alt[0].out_buf;
          e = launch_lh_fused(f, s);
          break;
        }
        HApplyLaunch h{};
        h.t = inter;
        h.nmax = st.nmax;
        h.tasks = reinterpret_cast<const HTask*>(blob + st.off0);
        h.planes = reinterpret_cast<const HPlane*>(blob + st.off1);
        h.work = reinterpret_cast<const HWork*>(blob + st.off2);
        h.nwork = st.n0;
        h.ptrs = dptrs;
        h.coef = inter == ElemType::F64 ? (const void*)(wsb + P.ws_coef64_off)
                                        : (const void*)(wsb + P.ws_coef32_off);
        h.off32 = st.mpo_off32;
        if (planes && st.has_alt) {
          h.np = np == 1 ? 0 : np;   // float64 panels: plain float64 outputs
          h.tasks = reinterpret_cast<const HTask*>(blob + st.off3);
          h.planes = reinterpret_cast<const HPlane*>(blob + st.off4);
          h.off32 = st.mpo_off32_alt;
          if (h.np > 0) {   // bfloat16 planes out: the XCD-grouped item order
            h.work = reinterpret_cast<const HWork*>(blob + st.off5);
            h.nwork = st.n1;
          }
        }
        if (P.sparse_mpo) {
          h.cnt = reinterpret_cast<const int32_t*>(wsb + P.ws_cnt_off);
          h.idx = reinterpret_cast<const int32_t*>(wsb + P.ws_idx_off);
          h.val = inter == ElemType::F64 ? (const void*)(wsb + P.ws_val64_off)
                                         : (const void*)(wsb + P.ws_val32_off);
        }
        e = launch_happly(h, s);
        break;
      }
    }
    check_hip(e, st.name.c_str());
    if (ev) check_hip(hipEventRecord((*ev)[k].second, s), "event");
  }
}

void run_steps(PlanData& P, void* ws, void* const* dptrs, bst_precision prec, hipStream_t s,
               bool skip_const, std::vector<std::pair<hipEvent_t, hipEvent_t>>* ev) {
  run_steps_impl(P, ws, dptrs, prec, s, skip_const, -1, ev);
}

static void drop_graph(PlanData& P) {
  if (P.gexec) (void)hipGraphExecDestroy(P.gexec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P.gexec = nullptr;
  P.graph = nullptr;
  P.graph_ws = nullptr;
}

static std::string tune_key(const PlanData& P, const Step& st, int form) {
  // structure signature: problem sizes and segment counts
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  mix((uint64_t)form);
  mix((uint64_t)st.transb);
  const bool alt = form >= 10 && st.has_alt;   // plane variant keys (10 + form)
  for (const auto& p : alt ? st.probs_alt : st.probs) {
    mix((uint64_t)p.M);
    mix((uint64_t)p.N);
    mix((uint64_t)p.seg_count);
  }
  for (const auto& g : alt ? st.segs_alt : st.segs) mix((uint64_t)g.K);
  (void)P;
  std::ostringstream os;
  os << st.name << "-" << std::hex << h;
  return os.str();
}

// A cached tile choice: the shape's fields (kind and stages may be absent
// in older files: kind 0).
struct CachedShape {
  int bm = 0, bn = 0, direct = 0, stages = 0;
  bool matches(const TileShape& s) const {
    return s.bm == bm && s.bn == bn && s.direct == direct && s.stages == stages;
  }
};

static std::map<std::string, CachedShape> load_cache(const char* path) {
  std::map<std::string, CachedShape> m;
  std::ifstream f(path);
  std::string line;
  // one entry per line: "key": [bm, bn, kind, stages],
  while (std::getline(f, line)) {
    auto q1 = line.find('"');
    auto q2 = line.find('"', q1 + 1);
    auto b1 = line.find('[');
    if (q1 == std::string::npos || q2 == std::string::npos || b1 == std::string::npos) continue;
    CachedShape c;
    if (std::sscanf(line.c_str() + b1, "[%d, %d, %d, %d]", &c.bm, &c.bn, &c.direct, &c.stages) >= 2)
      m[line.substr(q1 + 1, q2 - q1 - 1)] = c;
  }
  return m;
}

static void save_cache(const char* path, const std::map<std::string, CachedShape>& m) {
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : m) {
    f << "  \"" << kv.first << "\": [" << kv.second.bm << ", " << kv.second.bn << ", " << kv.second.direct
      << ", " << kv.second.stages << "]" << (++i < m.size() ? "," : "") << "\n";
  }
  f << "}\n";
}

// Cache entries of the variant choices, keyed by the plan's first GEMM step:
// FP64 float64 panels or per-block-pair kernels ([1, 0, 0, 0] for panels),
// and the fused L.psi + MPO kernel for the two-plane forms ([1, 0, 0, 0]
// when fused).
constexpr int kVariantKey = 99, kFusedKey = 98;
static std::string variant_key(const PlanData& P, int which = kVariantKey) {
  for (const auto& st : P.steps)
    if (st.kind == StepKind::Gemm) return tune_key(P, st, which);
  return std::string();
}

// Applies cached tile choices (if BST_TUNE_CACHE names a readable file).
void apply_tune_cache(PlanData& P) {
  const char* path = std::getenv("BST_TUNE_CACHE");
  if (!path) return;
  auto m = load_cache(path);
  const std::string vk = variant_key(P);
  if (!vk.empty()) {
    auto it = m.find(vk);
    if (it != m.end()) P.fp64_panels_on = it->second.bm != 0;
    auto itf = m.find(variant_key(P, kFusedKey));
    if (itf != m.end()) P.fused_on = itf->second.bm != 0;
  }
  for (auto& st : P.steps) {
    if (st.kind != StepKind::Gemm) continue;
    for (int f : {0, 1, 2, 3, 10, 12, 13}) {
      auto it = m.find(tune_key(P, st, f));
      if (it == m.end()) continue;
      const auto& shapes = f >= 10 ? gemm_planes_shapes(plane_count_of_key(f)) : gemm_tile_shapes((bst_precision)f);
      for (size_t i = 0; i < shapes.size(); ++i)
        if (it->second.matches(shapes[i])) st.tile_choice[f] = (int)i;
    }
  }
}

}  // namespace bst

using namespace bst;

extern "C" {

bst_status bst_plan_use_graph(bst_plan* p, int32_t on) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  p->p.use_graph = on != 0;
  if (!on) drop_graph(p->p);
  BST_CATCH
}

bst_status bst_execute(bst_plan* p, const void* const* in, void* const* out, void* ws,
                       void* stream) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  PlanData& P = p->p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  check_hip(hipGetLastError(), "pending device error");
  void* dptrs = prepare_ws(P, in, out, ws, s);
  if (!P.use_graph) {
    run_steps(P, ws, static_cast<void* const*>(dptrs), P.prec, s, false);
  } else {
    if (!P.gexec || P.graph_ws != ws || P.graph_prec != P.prec) {
      drop_graph(P);
      hipStream_t cs;
      check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        check_hip(e, "begin capture");
      }
      try {
        run_steps(P, ws, static_cast<void* const*>(dptrs), P.prec, cs, false);
      } catch (...) {
        hipGraph_t g;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        throw;
      }
      e = hipStreamEndCapture(cs, &P.graph);
      (void)hipStreamDestroy(cs);
      check_hip(e, "end capture");
      check_hip(hipGraphInstantiate(&P.gexec, P.graph, nullptr, nullptr, 0), "graph instantiate");
      P.graph_ws = ws;
      P.graph_prec = P.prec;
    }
    check_hip(hipGraphLaunch(P.gexec, s), "graph launch");
  }
  BST_CATCH
}

}  // extern "C"

namespace bst {
// Workspace of bst_execute_static: a fixed device array instead of caller
// memory, for callers that cannot allocate.  Each device holds its own copy;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device, fetched once per device on that device's first
// call.  Every call on a device shares its copy.
static __device__ __align__(256) unsigned char scratch[BST_STATIC_WORKSPACE_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static void* scratch_address() {
  int dev = -1;
  check_hip(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kMaxDevices) fail(BST_E_DEVICE, "device index out of range for the static workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static workspace address");
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0) fail(BST_E_DEVICE, "static workspace misaligned");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace bst

extern "C" {

bst_status bst_execute_static(bst_plan* p, const void* const* in, void* const* out, void* stream) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  PlanData& P = p->p;
  if (P.ws_bytes > (size_t)BST_STATIC_WORKSPACE_BYTES)
    fail(BST_E_INVALID, "plan needs " + std::to_string(P.ws_bytes) + " bytes of workspace; the static "
                        "workspace holds " + std::to_string((size_t)BST_STATIC_WORKSPACE_BYTES));
  hipStream_t s = static_cast<hipStream_t>(stream);
  check_hip(hipGetLastError(), "pending device error");
  void* ws = scratch_address();
  // tables go up again if another plan used this device's copy since
  void* dptrs = prepare_ws(P, in, out, ws, s);
  run_steps(P, ws, static_cast<void* const*>(dptrs), P.prec, s, false);
  BST_CATCH
}

bst_status bst_plan_profile(bst_plan* p, const void* const* in, void* const* out, void* ws,
                            void* stream, int32_t reps, double* step_ms, int32_t cap,
                            int32_t* nsteps) {
  BST_TRY
  if (!p || !step_ms || !nsteps) fail(BST_E_INVALID, "null argument");
  PlanData& P = p->p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* dptrs = prepare_ws(P, in, out, ws, s);
  const size_t n = P.steps.size();
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev(n);
  for (auto& e : ev) {
    check_hip(hipEventCreate(&e.first), "event");
    check_hip(hipEventCreate(&e.second), "event");
  }
  std::vector<double> acc(n, 0.0);
  reps = std::max(reps, 1);
  for (int r = 0; r < reps; ++r) {
    run_steps(P, ws, static_cast<void* const*>(dptrs), P.prec, s, false, &ev);
    check_hip(hipStreamSynchronize(s), "profile sync");
    for (size_t k = 0; k < n; ++k) {
      if (!step_runs(P, P.steps[k], P.prec, false)) continue;
      float ms = 0;
      check_hip(hipEventElapsedTime(&ms, ev[k].first, ev[k].second), "event time");
      acc[k] += ms;
    }
  }
  for (auto& e : ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  *nsteps = (int32_t)n;
  for (size_t k = 0; k < n && (int)k < cap; ++k) step_ms[k] = acc[k] / reps;
  BST_CATCH
}

bst_status bst_plan_autotune(bst_plan* p, const void* const* in, void* const* out, void* ws,
                             void* stream, int32_t reps) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  PlanData& P = p->p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  reps = std::max(reps, 1);
  void* dptrs = prepare_ws(P, in, out, ws, s);
  void* const* table = static_cast<void* const*>(dptrs);
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "event");
  check_hip(hipEventCreate(&e1), "event");
  const char* path = std::getenv("BST_TUNE_CACHE");
  auto cache = path ? load_cache(path) : std::map<std::string, CachedShape>{};
  const bst_precision form = P.prec;
  // A buffer twice the size of the last-level cache, rewritten before every
  // timed run: an iterative caller (Lanczos) streams its basis between two
  // applies, so no operand of one apply is still cached at the next.
  struct Flush {
    double* p = nullptr;
    hipStream_t s = nullptr;
    ~Flush() {
      if (!p) return;
      (void)hipStreamSynchronize(s);
      (void)hipFree(p);
    }
  } flush;
  flush.s = s;
  constexpr int64_t kFlushDoubles = (int64_t)64 << 20;   // 512 MiB
  if (hipMalloc(&flush.p, sizeof(double) * kFlushDoubles) != hipSuccess) {
    flush.p = nullptr;
    (void)hipGetLastError();
  } else {
    check_hip(hipMemsetAsync(flush.p, 0, sizeof(double) * kFlushDoubles, s), "flush buffer");
  }
  // reps runs of step k (all steps for k < 0), each after a cache flush and
  // the (untimed) steps before k, in ms
  auto time_runs = [&](int k) {
    double total = 0.0;
    for (int r = 0; r < reps; ++r) {
      if (flush.p) check_hip(launch_cache_flush(flush.p, kFlushDoubles, s), "cache flush");
      for (int j = 0; j < k; ++j) run_steps_impl(P, ws, table, P.prec, s, true, j, nullptr);
      check_hip(hipEventRecord(e0, s), "event");
      // a whole apply as an iterative caller repeats it: steps on constant
      // operands (their splits, copies) ran once before and are not timed
      run_steps_impl(P, ws, table, P.prec, s, k < 0, k, nullptr);
      check_hip(hipEventRecord(e1, s), "event");
      check_hip(hipEventSynchronize(e1), "event sync");
      float ms = 0;
      check_hip(hipEventElapsedTime(&ms, e0, e1), "event time");
      total += ms;
    }
    return total;
  };
  // the fastest tile shape of every GEMM step, in the variant the plan runs
  // now.  Each candidate is timed in the state an iterative caller leaves
  // (caches flushed, then the steps before it run): a step timed in a loop
  // finds its inputs in the caches, which favours shapes that re-read them.
  auto tune_steps = [&]() {
    // one full run so that intermediates hold realistic data
    run_steps(P, ws, table, P.prec, s, false);
    for (size_t k = 0; k < P.steps.size(); ++k) {
      Step& st = P.steps[k];
      if (st.kind != StepKind::Gemm) continue;
      const bst_precision f = st.fixed_fp64 ? BST_FP64 : form;
      const bool pl = uses_planes(P, form) && st.has_alt;
      const int key = pl ? planes_key(form) : (int)f;
      const auto& shapes = pl ? gemm_planes_shapes(plane_count(form)) : gemm_tile_shapes(f);
      double best = 1e30;
      int best_i = pl ? planes_tile(st, form) : default_tile(st, f);
      for (size_t i = 0; i < shapes.size(); ++i) {
        st.tile_choice[key] = (int)i;
        run_steps_impl(P, ws, table, P.prec, s, false, (int)k, nullptr);
        const double ms = time_runs((int)k);
        if (ms < best) {
          best = ms;
          best_i = (int)i;
        }
      }
      st.tile_choice[key] = best_i;
      const TileShape& bs = shapes[best_i];
      cache[tune_key(P, st, key)] = {bs.bm, bs.bn, bs.direct, bs.stages};
    }
  };
  // FP64 with padded layouts available: tune both variants (per-block-pair
  // kernels, float64 panels) and keep the one whose whole apply is faster,
  // unless an environment override fixes the variant
  const bool both = form == BST_FP64 && P.has_planes && P.f64_panels && !std::getenv("BST_FP64_BLOCKS") &&
                    !std::getenv("BST_FP64_PANELS");
  if (both) {
    P.fp64_panels_on = false;
    tune_steps();
    const double t_blocks = time_runs(-1);
    P.fp64_panels_on = true;
    tune_steps();
    const double t_panels = time_runs(-1);
    P.fp64_panels_on = t_panels < t_blocks;
    const std::string vk = variant_key(P);
    if (!vk.empty()) cache[vk] = {P.fp64_panels_on ? 1 : 0, 0, 0, 0};
  } else if (P.fused_ok && uses_planes(P, form) && plane_count(form) == 2 && !std::getenv("BST_FUSED_MPO")) {
    // two-plane form with a fused schedule: tune the GEMM tiles unfused, then
    // keep the fused L.psi + MPO kernel if the whole apply is faster with it
    P.fused_on = false;
    tune_steps();
    const double t_split = time_runs(-1);
    P.fused_on = true;
    const double t_fused = time_runs(-1);
    P.fused_on = t_fused < t_split;
    const std::string fk = variant_key(P, kFusedKey);
    if (!fk.empty()) cache[fk] = {P.fused_on ? 1 : 0, 0, 0, 0};
  } else {
    tune_steps();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(P);
  if (path) save_cache(path, cache);
  BST_CATCH
}

bst_status bst_plan_record_tiles(const bst_plan* p) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  const char* path = std::getenv("BST_TUNE_CACHE");
  if (!path) fail(BST_E_INVALID, "BST_TUNE_CACHE is not set");
  const PlanData& P = p->p;
  auto cache = load_cache(path);
  const std::string vk = variant_key(P);
  if (!vk.empty() && P.f64_panels) cache[vk] = {P.fp64_panels_on ? 1 : 0, 0, 0, 0};
  for (const auto& st : P.steps) {
    if (st.kind != StepKind::Gemm) continue;
    for (const auto& kv : st.tile_choice) {
      const int key = kv.first;
      const auto& shapes = key >= 10 ? gemm_planes_shapes(plane_count_of_key(key)) : gemm_tile_shapes((bst_precision)key);
      if (kv.second < 0 || kv.second >= (int)shapes.size()) continue;
      const TileShape& bs = shapes[kv.second];
      cache[tune_key(P, st, key)] = {bs.bm, bs.bn, bs.direct, bs.stages};
    }
  }
  save_cache(path, cache);
  BST_CATCH
}

static const std::vector<TileShape>& variant_list(const PlanData& P, bst_precision form, bool& planes) {
  planes = uses_planes(P, form);
  return planes ? gemm_planes_shapes(plane_count(form)) : gemm_tile_shapes(form);
}

bst_status bst_plan_tile_count(const bst_plan* p, bst_precision form, int32_t* count) {
  BST_TRY
  if (!p || !count) fail(BST_E_INVALID, "null argument");
  if (form < BST_FP64 || form > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  bool pl;
  *count = (int32_t)variant_list(p->p, form, pl).size();
  BST_CATCH
}

bst_status bst_plan_set_tile(bst_plan* p, bst_precision form, int32_t tile) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  if (form < BST_FP64 || form > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  PlanData& P = p->p;
  bool pl;
  const auto& list = variant_list(P, form, pl);
  if (tile < 0 || tile >= (int32_t)list.size()) fail(BST_E_INVALID, "tile index out of range");
  for (auto& st : P.steps) {
    if (st.kind != StepKind::Gemm) continue;
    if (pl && st.has_alt) st.tile_choice[10 + (int)form] = tile;
    else if (!pl) st.tile_choice[(int)form] = tile;
  }
  drop_graph(P);
  BST_CATCH
}

bst_status bst_plan_forget_workspace(bst_plan* p) {
  BST_TRY
  if (!p) fail(BST_E_INVALID, "null plan");
  drop_graph(p->p);
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();) {
    if (it->second == p->p.id) it = g_ws_owner.erase(it);
    else ++it;
  }
  p->p.uploaded_ws = nullptr;
  p->p.last_ptrs.clear();
  BST_CATCH
}

bst_status bst_plan_destroy(bst_plan* p) {
  if (p) {
    drop_graph(p->p);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();) {
      if (it->second == p->p.id) it = g_ws_owner.erase(it);
      else ++it;
    }
  }
  delete p;
  set_last_error("");
  return BST_OK;
}

}  // extern "C"

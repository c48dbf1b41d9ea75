// Plans: the integer bookkeeping of a contraction (charge-sector matching,
// GEMM problem lists, permute jobs, MPO-apply tasks) and its execution.
#pragma once

#include "bst_internal.h"

struct bst_tensor {
  std::unique_ptr<bst::TensorDesc> d;
};

#define BST_TRY try {
#define BST_CATCH                                            \
  }                                                          \
  catch (const bst::Error& e) {                              \
    bst::set_last_error(e.msg);                              \
    return e.status;                                         \
  }                                                          \
  catch (const std::bad_alloc&) {                            \
    bst::set_last_error("host out of memory");               \
    return BST_E_INVALID;                                    \
  }                                                          \
  catch (const std::exception& e) {                          \
    bst::set_last_error(e.what());                           \
    return BST_E_INVALID;                                    \
  }                                                          \
  bst::set_last_error("");                                   \
  return BST_OK;

namespace bst {

const TensorDesc* desc_of(const bst_tensor* t);
bst_tensor* wrap_tensor(std::unique_ptr<TensorDesc> d);
void set_last_error(const std::string& s);

enum class StepKind { Permute, Gemm, HCoef, HApply, Split, Expand };

// Element type of a step operand: fixed, or the plan's intermediate type
// (float64 for BST_FP64, float32 for the other forms).
enum class Elem { F64, Inter };

struct Step {
  StepKind kind;
  std::string name;
  double flops = 0;   // algorithmic flops of this step
  double bytes = 0;   // algorithmic HBM bytes with float64 intermediates
  double bytes32 = 0; // the same with float32 intermediates
  // GEMM
  Elem ta = Elem::F64, tc = Elem::F64;
  bool transb = false;
  bool fixed_fp64 = false;   // always runs in BST_FP64 (packing-free exact steps)
  std::vector<GemmProb> probs;
  std::vector<GemmSeg> segs;
  std::map<int, int> tile_choice;   // form -> index into gemm_tile_shapes(form)
  // Permute
  std::vector<PermJob> jobs;
  std::vector<PermWork> pwork;
  // Expand (complex contraction)
  std::vector<ExpandJob> xjobs;
  std::vector<ExpandWork> xwork;
  // HCoef / HApply (paired: the apply uses the coefficients of the coef step)
  struct RawTerm {
    int32_t cls, o, i;
    HTerm t;
  };
  std::vector<RawTerm> terms;
  int32_t ncls = 0;
  int32_t nmax = 0;
  std::vector<HTask> tasks;
  std::vector<HPlane> planes;
  std::vector<int32_t> task_group;   // per task: its a sector (tasks of one a share T1 and T3 rows)
  // L.psi fused into the MPO apply (plane variant of an H_eff plan): per
  // input plane of tasks_alt, the GEMM that forms it (L rows of (a, w1)
  // against the transposed psi block (a', t1, t2, b'), K = g(a'); K = 0 for
  // T1 blocks no pair reaches), and task_fin[t] = first input of task t
  struct FusedIn {
    int64_t a_off, b_off;
    int32_t a_ld, b_ld, K, pad;
  };
  std::vector<FusedIn> fins;
  std::vector<int32_t> task_fin;
  bool fusable = false;              // an L.psi GEMM step the fused kernel replaces
  Elem th = Elem::Inter;
  // bfloat16-plane variant used by the split forms (H_eff only): GEMM
  // segments on pre-split operands, MPO tasks writing T3 as planes
  bool has_alt = false;
  std::vector<GemmProb> probs_alt;   // problems of the plane variant (may merge blocks)
  std::vector<int64_t> rowmap;       // C row offsets of probs_alt with rowmap1 > 0
  std::vector<GemmSeg> segs_alt;     // indexed by probs_alt[].seg_begin
  std::vector<HTask> tasks_alt;
  std::vector<HPlane> planes_alt;
  // Split (float64 -> bfloat16 planes), run only by the split forms
  std::vector<SplitJob> sjobs;
  std::vector<SplitWork> swork;
  // operand-only preparation, valid for as long as L, W and R do not change
  bool constant = false;
  // MPO apply: every plane index (scaled for the bfloat16 plane interleave)
  // has a byte offset below 2^32, so the kernel may index in 32 bits
  bool mpo_off32 = false, mpo_off32_alt = false;
  // the split of the H_eff input psi (reads float32 rows while the plan runs
  // inside a float32-basis Lanczos solve)
  bool reads_psi = false;
  // the GEMM that writes the H_eff output (float32 while the plan runs inside
  // a float32-basis Lanczos solve)
  bool writes_out = false;
  // device table offsets inside the plan blob (filled by finalize)
  size_t off0 = 0, off1 = 0, off2 = 0, off3 = 0, off4 = 0, off5 = 0;
  int64_t n0 = 0, n1 = 0;
  std::map<std::pair<int, int>, std::pair<size_t, int64_t>> tile_lists;  // (bm,bn) -> (off, n)
  std::map<std::pair<int, int>, std::pair<size_t, int64_t>> tile_lists_alt;  // plane variant
  // k-step schedules of the pipelined plane kernel, by np * 64 + shape index
  struct StreamList {
    bool ok = false;               // the problems fit the kernel's layout rules
    size_t steps_off = 0, begin_off = 0, rows_off = 0;
    int64_t nwg = 0;
  };
  std::map<int, StreamList> streams_alt;
  StreamList fused;                  // HApply: k-step schedule of the fused kernel
  size_t fused_planes_off = 0;       // tasks_alt planes with nmax spare records
};

struct InternalBuf {
  int32_t slot;
  size_t bytes;     // sized for float64
  size_t ws_off;
};

struct PlanData {
  int kind = 0;                 // 0 permute, 1 contract, 2 heff, 3 heff batch
  bst_precision prec = BST_FP64;
  std::vector<int32_t> in_slots, out_slots;
  std::vector<int64_t> in_numel, out_numel;   // elements per buffer (null allowed when 0)
  std::vector<InternalBuf> internals;
  int32_t nslots = 0;
  std::vector<Step> steps;
  // heff bookkeeping (single apply): psi numel for Lanczos
  int64_t psi_numel = 0;
  int64_t t1_numel = 0, t3_numel = 0;
  bool has_planes = false;      // split forms run the bfloat16-plane variant
  // every plane-variant GEMM step has a float64 k-step schedule, so FP64 can
  // run on float64 operands in the same padded layouts (finalize)
  bool f64_panels = false;
  // FP64 runs on the float64 panels (chosen by the autotuner when its whole
  // apply is faster than with the per-block-pair kernels)
  bool fp64_panels_on = false;
  bool fused_ok = false;             // an MPO step has a fused schedule (two-plane forms)
  bool fused_on = false;             // run it (autotuner choice, BST_FUSED_MPO overrides)
  bool sparse_mpo = true;       // MPO apply runs only the nonzero h entries
  // finalize
  std::vector<uint8_t> blob;
  size_t ws_ptr_off = 0, ws_blob_off = 0, ws_coef64_off = 0, ws_coef32_off = 0, ws_bytes = 0;
  size_t ws_cnt_off = 0, ws_idx_off = 0, ws_val64_off = 0, ws_val32_off = 0;
  int32_t coef_entries = 0;
  bool finalized = false;
  // execution state
  bool use_graph = false;
  bool psi_f32 = false;         // set by Lanczos: the psi input is a float32 Krylov row
  bool z_f32 = false;           // set by Lanczos: the output H psi is written as float32
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  void* graph_ws = nullptr;
  bst_precision graph_prec = BST_FP64;
  std::vector<void*> last_ptrs;
  void* uploaded_ws = nullptr;
  uint64_t id = 0;
};

void finalize(PlanData& p);
// Uploads tables (if this plan's tables are not in ws yet) and the pointer
// table built from in / out; returns the device address of the pointer table.
void* prepare_ws(PlanData& p, const void* const* in, void* const* out, void* ws, hipStream_t s);
// Uploads an extra pointer table at ws + off (Lanczos) and returns it.
void* upload_table(PlanData& p, const std::vector<void*>& ptrs, void* ws, size_t off,
                   hipStream_t s);
std::vector<void*> build_ptrs(PlanData& p, const void* const* in, void* const* out, void* ws);
// Enqueues the plan's kernels with the given device pointer table.
// skip_const: leave out the steps that depend only on L, W and R (their
// results from an earlier execute on the same workspace are still valid).
void run_steps(PlanData& p, void* ws, void* const* dptrs, bst_precision prec, hipStream_t s,
               bool skip_const, std::vector<std::pair<hipEvent_t, hipEvent_t>>* ev = nullptr);
// The padded-layout variant runs for this form: bfloat16 planes for the
// split forms; float64 operands for FP64 when the autotuner chose them or
// BST_FP64_PANELS is set (BST_FP64_BLOCKS keeps FP64 on the per-block-pair
// kernels).
bool uses_planes(const PlanData& p, bst_precision prec);
// Planes of the padded-layout variant of a form: 1 (float64), 2 or 3.
int plane_count(bst_precision prec);
// Plane count of a tile-choice key of the padded-layout variant (10 + form).
int plane_count_of_key(int key);
bool step_runs(const PlanData& p, const Step& st, bst_precision prec, bool skip_const);
bool fused_active(const PlanData& p, bst_precision prec);
int planes_tile(const Step& st, bst_precision prec);
int default_tile(const Step& st, bst_precision form);
void run_steps_impl(PlanData& p, void* ws, void* const* dptrs, bst_precision prec, hipStream_t s,
                    bool skip_const, int only_step,
                    std::vector<std::pair<hipEvent_t, hipEvent_t>>* ev);
// Applies tile choices recorded by the autotuner (file named by BST_TUNE_CACHE).
void apply_tune_cache(PlanData& p);

}  // namespace bst

struct bst_plan {
  bst::PlanData p;
};

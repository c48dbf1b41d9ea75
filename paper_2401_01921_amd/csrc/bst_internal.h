// Internal types of the block-sparse library: host descriptors, plan tables
// and the device-side records the kernels read.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/bst.h"

namespace bst {

// Device pointers taken from a plan's pointer table address global memory;
// declaring that (address space 1) lets the compiler emit global rather than
// flat memory instructions, whose completion is tracked apart from scalar
// loads (a flat access also holds up every wait for a scalar load).
#define BST_G __attribute__((address_space(1)))

// ------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------
struct Error {
  bst_status status;
  std::string msg;
};
[[noreturn]] void fail(bst_status s, const std::string& msg);
void check_hip(hipError_t e, const char* what);

// ------------------------------------------------------------------------
// Tensor descriptor (host only)
// ------------------------------------------------------------------------
// Charges of a leg: one component per symmetry.  `sym` holds the moduli
// (0: U(1), n >= 2: Z_n; empty: a single U(1) component); `q` is the first
// component of every sector and `qx` the others, (sym.size() - 1) per sector.
struct LegDesc {
  int32_t dir = 1;
  std::vector<int32_t> q;
  std::vector<int32_t> qx;
  std::vector<int32_t> sym;
  std::vector<int64_t> g;
  std::string label;
  int64_t total() const {
    int64_t s = 0;
    for (auto v : g) s += v;
    return s;
  }
  int nsym() const { return sym.empty() ? 1 : (int)sym.size(); }
  int32_t modulus(int c) const { return sym.empty() ? 0 : sym[c]; }
  int32_t charge(int sector, int c) const {
    return c == 0 ? q[sector] : qx[(size_t)sector * (nsym() - 1) + (c - 1)];
  }
  bool same_charges(const LegDesc& o) const { return q == o.q && qx == o.qx && sym == o.sym; }
  bool same_sectors(const LegDesc& o) const { return same_charges(o) && g == o.g; }
};

struct TensorDesc {
  std::vector<LegDesc> legs;
  int64_t nblocks = 0;
  int64_t numel = 0;
  std::vector<int32_t> qn;      // nblocks * rank sector indices
  std::vector<int64_t> shape;   // nblocks * rank
  std::vector<int64_t> offset;  // nblocks
  std::unordered_map<std::string, int64_t> lookup;

  int rank() const { return (int)legs.size(); }
  // Enumerates the valid blocks in canonical order (called once by create).
  void build();
  // Block index of a sector tuple, -1 if it is not a valid block.
  int64_t find(const int32_t* t) const;
  const int32_t* block_qn(int64_t b) const { return qn.data() + b * rank(); }
  const int64_t* block_shape(int64_t b) const { return shape.data() + b * rank(); }
  int64_t block_size(int64_t b) const {
    int64_t n = 1;
    for (int i = 0; i < rank(); ++i) n *= block_shape(b)[i];
    return n;
  }
  int label_index(const std::string& l) const;
};

std::unique_ptr<TensorDesc> make_tensor(std::vector<LegDesc> legs);

// ------------------------------------------------------------------------
// Device records
// ------------------------------------------------------------------------
// One K-segment of a grouped-GEMM problem.  A is [M x K] row-major with
// leading dim lda; B is [K x N] (ldb) or, for transposed-B steps, [N x K].
// For bfloat16-plane operands these are planar positions (see plane_at).
struct GemmSeg {
  int64_t a_off, b_off;
  int32_t a_buf, b_buf;
  int32_t K, lda, ldb, pad;
};

// bfloat16 planes of a split operand are interleaved by 8-element chunks.
// An operand is laid out by planar positions (block offset + row * ld + k,
// ld a multiple of 32); with np planes, plane q of position pos is stored
// at element
//   np * (pos - pos % 8) + 8 * q + pos % 8,
// so one 32-deep k step of one row, all planes, is 64 * np contiguous
// bytes: a whole 128-byte line for np = 2 (rows start on 32-element bounds),
// which the memory system fetches as one request instead of two.
__host__ __device__ constexpr int64_t plane_at(int np, int64_t pos, int q) {
  return np * (pos - (pos & 7)) + 8 * q + (pos & 7);
}
// The same in 32 bits, for callers that checked that the result fits.
__host__ __device__ constexpr uint32_t plane_at(int np, uint32_t pos, int q) {
  return (uint32_t)np * (pos - (pos & 7u)) + 8u * (uint32_t)q + (pos & 7u);
}
// One output block: C[M x N] row-major (ldc) = sum over its segments.
struct GemmProb {
  int64_t c_off;
  int32_t c_buf, M, N, ldc;
  int32_t seg_begin, seg_count;
  // 0: row r of C starts at c_off + r*ldc.  Otherwise (plane kernels only)
  // row r starts at rowmap[rowmap1 - 1 + r], an element offset into the
  // C buffer: the rows of one problem may belong to several output blocks.
  int32_t rowmap1, pad;
};
struct GemmTile {
  int32_t prob, m0, n0, pad;
};

// Block permute job: one block, row-major input shape and, per input dim,
// the stride of that dim in the output block.
constexpr int kMaxRank = 8;
struct PermJob {
  int64_t in_off, out_off;
  int32_t in_buf, out_buf;
  int32_t rank;
  int32_t pdim;       // input dim that is fastest in the output (tile jobs)
  int32_t shape[kMaxRank];
  int64_t istride[kMaxRank];
  int64_t ostride[kMaxRank];
};
// A work item of the permute kernels: a tile (transposing jobs) or a row
// range (jobs that keep the fastest dim).
constexpr int kPermRows = 1024;   // most rows in one row-copy work item
struct PermWork {
  int32_t job;
  int32_t kind;       // 0: rows; 1, 2, 3: a 64 x 64, 128 x 32 or 256 x 16 tile
  int64_t batch;      // rows: first row; tile: linear index over batch dims
  int32_t t0, t1;     // tile origin along (p, last) or row count
};

// MPO (two-site h) apply: one (a-sector, b'-sector) pair of T1 / T3.
struct HTask {
  int32_t rows, cols;        // g_a, g_b'
  int32_t cls;               // coefficient class
  int32_t nin, nout;
  int32_t plane_begin;       // nin input planes then nout output planes
  int32_t in_buf, out_buf;
};

// Conversion of float64 blocks into bfloat16 planes with rows padded to a
// multiple of 32 elements: plane q of position out_off + r*out_ld + c (see
// plane_at) for r < rows, c < out_ld (zero beyond cols).  With transpose set, the block
// [rows x cols] is written as [cols x rows] (rows padded instead).
struct SplitJob {
  int64_t in_off, out_off;
  int32_t in_buf, out_buf;
  int32_t rows, cols, out_ld, transpose;
};
struct SplitWork {
  int32_t job, r0, c0, pad;
};
// A split work item with its job's fields copied in (the kernel's table:
// one dependent read fewer before the first data load).
struct SplitItem {
  int64_t in_off, out_off;
  int32_t in_buf, out_buf;
  int32_t rows, cols, out_ld, transpose;
  int32_t r0, c0;
};
struct HPlane {
  int64_t off;               // element offset of (row 0, col 0)
  int64_t rowstride;
};
struct HWork {
  int32_t task;
  int32_t site0;
};
// coef[cls][o][i] = sum of W1[w1] * W2[w2] over the entry's terms.
struct HTerm {
  int32_t w1_buf, w2_buf;
  int64_t w1_off, w2_off;
};

// ------------------------------------------------------------------------
// Kernel launchers (kernels_*.hip)
// ------------------------------------------------------------------------
enum class ElemType : int { F64 = 0, F32 = 1 };

struct TileShape {
  int bm, bn;
  int direct = 0;   // 1: LDS-free kernel (fragments loaded straight from memory);
                    // 3: pipelined persistent kernel on a k-step schedule (padded layouts only)
  int stages = 0;   // kind 3: LDS stages (copies run stages - 1 k-steps ahead)
  int waves = 4;    // kind 3: waves per workgroup (4: 2 x 2, or 1 x 4 for 192 columns; 8: 2 x 4, or 4 x 2 when bm > bn)
};
// Tile shapes compiled for each arithmetic form.
const std::vector<TileShape>& gemm_tile_shapes(bst_precision form);

struct GemmLaunch {
  bst_precision form;
  ElemType ta, tb, tc;
  bool transb;
  int tile;                    // index into gemm_tile_shapes(form)
  const GemmTile* tiles;
  const GemmProb* probs;
  const GemmSeg* segs;
  void* const* ptrs;
  int64_t ntiles;
};
hipError_t launch_gemm(const GemmLaunch& g, hipStream_t s);
hipError_t launch_gemm_direct(const GemmLaunch& g, int bm, int bn, hipStream_t s);

// Complex contraction: one block of B (complex, [K x N] with K the
// contracted and N the free extent) expanded into the real block
// [K x 2 x N x 2] = [[Br, Bi], [-Bi, Br]] per element, so that the real
// product of A's interleaved (re, im) rows with it gives C interleaved.
struct ExpandJob {
  int64_t in_off, out_off;   // float64 offsets
  int32_t in_buf, out_buf;
  int32_t K, N;
};
struct ExpandWork {
  int32_t job, start;        // 4096 complex elements of a job per workgroup
};
struct ExpandLaunch {
  const ExpandJob* jobs;
  const ExpandWork* work;
  void* const* ptrs;
  int64_t nwork;
};
hipError_t launch_expand(const ExpandLaunch& l, hipStream_t s);

struct PermLaunch {
  const PermJob* jobs;
  const PermWork* work;
  void* const* ptrs;
  int64_t nwork;
};
hipError_t launch_permute(const PermLaunch& p, hipStream_t s);

struct HCoefLaunch {
  const HTerm* terms;
  const int32_t* entry_begin;  // nentries + 1
  int64_t nentries;            // ncls * nmax * nmax
  int nmax;
  void* const* ptrs;
  double* coef64;
  float* coef32;
  // compacted rows: cnt[ncls*nmax], idx / val[ncls*nmax*nmax]
  int32_t* cnt;
  int32_t* idx;
  double* val64;
  float* val32;
};
hipError_t launch_hcoef(const HCoefLaunch& c, hipStream_t s);

struct SplitLaunch {
  int np;
  bool in_f32 = false;         // the input blocks are float32 (a float32 Krylov row)
  const SplitItem* items;
  void* const* ptrs;
  int64_t nwork;
};
hipError_t launch_split(const SplitLaunch& l, hipStream_t s);

// Grouped GEMM on pre-split bfloat16 planes (layout: plane_at): A [M x K]
// and B [N x K], both with K contiguous, float32 accumulate.
struct PlanesLaunch {
  int np;                      // 2 (BF16X3) or 3 (BF16X6)
  ElemType tc;
  int tile;                    // index into gemm_planes_shapes(np)
  const GemmTile* tiles;
  const GemmProb* probs;
  const GemmSeg* segs;
  void* const* ptrs;
  int64_t ntiles;
  const int64_t* rowmap = nullptr;   // row offsets of problems with rowmap1 > 0
};
const std::vector<TileShape>& gemm_planes_shapes(int np);
hipError_t launch_gemm_planes(const PlanesLaunch& g, hipStream_t s);

// Pipelined plane GEMM (kernels_stream.hip).  The host lists, for every
// workgroup of a fixed grid, the 32-deep k-steps of the output tiles it
// owns, one 48-byte record per step, the steps of a tile consecutive.
// A tile row r < rows reads plane q of A at planar position a + r*lda + k, B likewise;
// chunks of 8 k at or past kch read as zero and chunk kch-1 holds kval valid
// elements.  With float64 operands (np = 1) a step is 16 deep and its
// "chunks" are 16-byte pieces of two elements (kch 0..8, kval 1..2).  The last step of a tile writes it: row r, column j to
// C[c + r*ldc + j] or, row-mapped, to C[rowtab[c + r] + j] (entries < 0
// skipped), for j < cols.
struct KStep {
  int64_t a, b;           // element offsets (plane 0) of tile row 0 at this k
  int32_t lda, ldb;
  uint8_t rows1, cols1;   // valid tile rows / columns minus one (0..bm-1, 0..bn-1)
  uint8_t kch;            // 8-element k chunks read from memory (0..4)
  uint8_t flags;          // kStepFirst | kStepLast | kStepRowmap
  uint8_t kval, pad;      // valid elements of chunk kch - 1 (1..8)
  uint16_t c_buf;         // pointer-table slots of C, A and B
  int64_t c;              // C offset of (row 0, col 0), or rowtab index of row 0
  int32_t ldc;
  uint16_t a_buf, b_buf;
};
static_assert(sizeof(KStep) == 48, "k-step record is 48 bytes");
constexpr int kStepFirst = 1, kStepLast = 2, kStepRowmap = 4;
constexpr int kStepPlaneEnd = 8;   // fused L.psi + MPO: last k-step of an input channel
constexpr int kStepBatch = 16;   // records copied into LDS per batch
constexpr int kStepRing = 3;     // batches resident in LDS
// LDS bytes of one workgroup of the pipelined kernel and workgroups per CU
// np = 1 names float64 operands (one plane of doubles): a 16-deep k-step of a
// row is 128 bytes, like a 32-deep step of two bfloat16 planes.
constexpr int stream_row_bytes(int np) { return np == 1 ? 128 : np * 64; }
constexpr int stream_lds_bytes(int np, int bm, int bn, int stages) {
  return stages * (bm + bn) * stream_row_bytes(np) + kStepRing * kStepBatch * 48 + stages * bm * 8;
}
constexpr int stream_wgs_per_cu(int np, int bm, int bn, int stages) {
  return 163840 / stream_lds_bytes(np, bm, bn, stages) < 1   ? 1
         : 163840 / stream_lds_bytes(np, bm, bn, stages) > 4 ? 4
                                                             : 163840 / stream_lds_bytes(np, bm, bn, stages);
}
constexpr int kStreamCUs = 256;   // compute units the schedule is balanced for

struct StreamLaunch {
  int np;                         // 2, 3: bfloat16 planes; 1: float64 operands
  ElemType tc;
  int tile;                       // index into gemm_planes_shapes(np), a kind-3 shape
  const KStep* steps;             // padded with kStepBatch records past the last
  const int64_t* wg_begin;        // nwg + 1 entries
  int64_t nwg;
  void* const* ptrs;
  const int64_t* rowtab;          // row offsets of row-mapped tiles (bm per tile)
};
hipError_t launch_gemm_planes_stream(const StreamLaunch& g, hipStream_t s);

// L.psi fused with the two-site MPO apply for two bfloat16 planes: 64 x 64
// tiles of the MPO tasks on 8 waves, one workgroup per CU.  Records as for
// the pipelined GEMM (see lh_fused_kernel for the fields it reuses).
constexpr int lh_fused_lds_bytes(int nmax) {
  return 3 * (64 + 64) * 128 + kStepRing * kStepBatch * 48 + 3 * (nmax * nmax * 4 + nmax * 16);
}
struct LhFusedLaunch {
  int nmax;                       // 8 or 16: the coefficient block is nmax x nmax floats
  const KStep* steps;             // padded with kStepBatch records past the last
  const int64_t* wg_begin;        // nwg + 1 entries
  int64_t nwg;
  void* const* ptrs;
  const float* coef;              // dense float32 coefficients [class][o][i]
  const HPlane* planes;           // task planes, nmax spare records at the end
  int out_slot;                   // pointer-table slot of the T3 planes
};
hipError_t launch_lh_fused(const LhFusedLaunch& f, hipStream_t s);

struct HApplyLaunch {
  int np = 0;                  // > 0: outputs written as np bfloat16 planes
  ElemType t;
  int nmax;
  const HTask* tasks;
  const HPlane* planes;
  const HWork* work;
  int64_t nwork;
  void* const* ptrs;
  const void* coef;            // double or float [ncls][nmax][nmax]
  // compacted nonzero coefficients (sparse kernel, nmax <= 16); null: dense
  const int32_t* cnt = nullptr;
  const int32_t* idx = nullptr;
  const void* val = nullptr;
  bool off32 = false;          // every plane index fits 32-bit byte offsets (plan-checked)
};
hipError_t launch_happly(const HApplyLaunch& h, hipStream_t s);
hipError_t launch_happly_sparse(const HApplyLaunch& h, hipStream_t s);

// Lanczos vector kernels (float64).  Reductions are deterministic: every
// block reduces a fixed element range in a fixed order into `partial`
// ([kVecBlocks][nvals]) and one more kernel adds the partials in order.
constexpr int kVecBlocks = 2048;
constexpr int kMaxVecs = 128;   // vectors handled by the fused kernels
// out[k] = sum_i V[k*ldv + i] w[i], k < nv
hipError_t launch_multidot(const double* V, int64_t ldv, int64_t n, int nv, const double* w,
                           double* partial, double* out, hipStream_t s);
// wout[i] = w[i] - sum_k V[k*ldv+i] c[k]  (wout may equal w), then
// mode 1: out[k] = sum_i V[k*ldv+i] wout[i] (k < nv)
// mode 2: out[0] = |wout|^2
hipError_t launch_project(const double* V, int64_t ldv, int64_t n, int nv, const double* c,
                          const double* w, double* wout, int mode, double* partial, double* out,
                          hipStream_t s);
// dst[i] = src[i] / sqrt(norm2[0]) (0 if norm2 <= 0); norm2 read on device.
hipError_t launch_scale_rnorm(const double* src, const double* norm2, double* dst, int64_t n,
                              hipStream_t s);
hipError_t launch_scale_rnorm(const double* src, const double* norm2, float* dst, int64_t n,
                              hipStream_t s);
// y[i] = sum_k coef[k] V[k*ldv+i]  (coef on device)
hipError_t launch_combine(const double* V, int64_t ldv, int64_t n, int nv, const double* coef,
                          double* y, hipStream_t s);
hipError_t launch_combine(const float* V, int64_t ldv, int64_t n, int nv, const double* coef,
                          double* y, hipStream_t s);
// out[0] = x.y, out[1] = y.y (out == nullptr: block partials only)
// Reads n doubles (zeros) with ordinary cached loads, so that data an earlier
// kernel left in the L2 and last-level caches is evicted.
hipError_t launch_cache_flush(double* buf, int64_t n, hipStream_t s);
hipError_t launch_dot2(const double* x, const double* y, int64_t n, double* partial, double* out,
                       hipStream_t s);
hipError_t launch_dot2(const float* x, const double* y, int64_t n, double* partial, double* out,
                       hipStream_t s);
// e = num[0]/num[1]; out[0] = |hy - e y|^2
hipError_t launch_resid(const double* hy, const double* y, const double* num, int64_t n,
                        double* partial, double* out, hipStream_t s);
// Reduces the pass-3 partials (grid of the project kernel for n elements),
// records alpha[j], beta[j], norm2_out[0] and writes vnext = w / beta_j
// (vnext may be null on the last step).  launch_project with out == nullptr
// leaves its partials unreduced for this kernel.
hipError_t launch_lanczos_step_end(const double* partial, int64_t n_for_grid, const double* c,
                                   const double* d, int j, double* alpha, double* beta,
                                   double* norm2_out, const double* w, double* vnext, int64_t n,
                                   hipStream_t s);
// One-pass Lanczos step j (see kernels_aux.hip).  The basis rows hold the
// residuals as the passes wrote them; cmat (kMaxVecs x kMaxVecs, row k at
// cmat + k * kMaxVecs, lower triangular) maps them to the orthonormal
// vectors, v_k = sum_{m<=k} C[k][m] u_m, and gains one row per step.
// dot step: from g = u_j.z (device scalar) and the previous pass's sums,
// dprev, alpha and beta of step j - 1, row j of C, and coef[0..j] (the
// coefficients of rows 0..j in the next residual) and aest.  pass: reads
// rows 0..j and z, writes the new residual to vnext (may be null), dn[0..j+1]
// = (u_m . w, w.w).  end: alpha[j], beta[j], dprev of the last step.
hipError_t launch_lanczos_pass(const double* V, int64_t ldv, int64_t n, int j, const double* z,
                               const double* coef, const double* beta, double* vnext, double* partial,
                               double* dn, hipStream_t s);
// The same with z in float32 (a split-form matvec's float32 accumulators,
// stored exactly).
hipError_t launch_lanczos_pass(const double* V, int64_t ldv, int64_t n, int j, const float* z,
                               const double* coef, const double* beta, double* vnext, double* partial,
                               double* dn, hipStream_t s);
// The same over a float32 basis (the residual rounded to float32 when
// written; dots and scalars in float64).
hipError_t launch_lanczos_pass(const float* V, int64_t ldv, int64_t n, int j, const float* z,
                               const double* coef, const double* beta, float* vnext, double* partial,
                               double* dn, hipStream_t s);
// The u_j.z dot and the scalar work of step j in two launches (dot partials,
// then one block that sums them and the partials of the pass of step j - 1,
// ends step j - 1 and forms row j of C and the scalars of step j); dn null
// in launch_lanczos_pass skips that pass's own sums, which this call (or
// launch_lanczos_pass_sums after the last step) then forms.
hipError_t launch_lanczos_dot_step(const double* x, const double* z, int64_t n, double* dpart,
                                   const double* ppart, int pj, double* dn, int j, double* g,
                                   double* alpha, double* beta, double* dprev, double* coef,
                                   double* aest, double* cmat, hipStream_t s);
hipError_t launch_lanczos_dot_step(const double* x, const float* z, int64_t n, double* dpart,
                                   const double* ppart, int pj, double* dn, int j, double* g,
                                   double* alpha, double* beta, double* dprev, double* coef,
                                   double* aest, double* cmat, hipStream_t s);
hipError_t launch_lanczos_dot_step(const float* x, const float* z, int64_t n, double* dpart,
                                   const double* ppart, int pj, double* dn, int j, double* g,
                                   double* alpha, double* beta, double* dprev, double* coef,
                                   double* aest, double* cmat, hipStream_t s);
hipError_t launch_lanczos_pass_sums(int64_t n, int j, bool f32, const double* partial, double* dn,
                                   hipStream_t s);
hipError_t launch_lanczos_end(const double* dn, const double* aest, int j, const double* cmat,
                              double* dprev, double* alpha, double* beta, hipStream_t s);
// alpha[j] = c[j] + d[j]; beta[j] = sqrt(norm2[0])
// plain device copy of n doubles

}  // namespace bst

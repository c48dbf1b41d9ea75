// Grouped sector GEMM without LDS: every lane loads its own MFMA operand
// fragments straight from global memory (L1/L2 catch the reuse between the
// waves of a workgroup), double-buffered in registers, with no barriers.
//
// Inside each chunk of 16 (float64/float32) or 32 (bfloat16) k values, lane
// group g = lane/16 owns a contiguous run of k (4g..4g+3, or 8g..8g+7), so a
// lane reads consecutive addresses of its row.  For the 16x16x4 MFMAs this
// permutes the order in which k enters the sum inside a chunk (a fixed
// permutation, so the results stay bitwise reproducible); for 16x16x32 it is
// the instruction's own layout.
#include "bst_internal.h"

namespace bst {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

template <int FORM, typename TA, typename TC, bool TRANSB, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_direct_kernel(const GemmTile* __restrict__ tiles,
                                                          const GemmProb* __restrict__ probs,
                                                          const GemmSeg* __restrict__ segs,
                                                          void* const* __restrict__ ptrs) {
  constexpr bool F64 = (FORM == BST_FP64);
  using CT = typename std::conditional<F64, double, float>::type;
  using ACC = typename std::conditional<F64, dbl4, flt4>::type;
  constexpr int WM = BM / 2, WN = BN / 2, SM = WM / 16, SN = WN / 16;

  const GemmTile t = tiles[blockIdx.x];
  if (t.prob < 0) return;   // padding of the per-XCD tile lists
  const GemmProb p = probs[t.prob];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int r16 = lane & 15, g4 = 4 * (lane >> 4);
  const int rbase = t.m0 + wm * WM + r16, cbase = t.n0 + wn * WN + r16;

  ACC acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = ACC{0, 0, 0, 0};

  CT a0[SM][4], b0[SN][4], a1[SM][4], b1[SN][4];
  int cs = 0, ck = 0;   // next (segment, k0) to load
  const int nseg = p.seg_count;

  auto load = [&](CT (&a)[SM][4], CT (&b)[SN][4]) {
    const GemmSeg sg = segs[p.seg_begin + cs];
    const BST_G TA* __restrict__ A = (const BST_G TA*)(ptrs[sg.a_buf]) + sg.a_off;
    const BST_G double* __restrict__ B = (const BST_G double*)(ptrs[sg.b_buf]) + sg.b_off;
#pragma unroll
    for (int i = 0; i < SM; ++i) {
      const int r = rbase + i * 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = ck + g4 + q;
        a[i][q] = (r < p.M && k < sg.K) ? (CT)A[(int64_t)r * sg.lda + k] : CT(0);
      }
    }
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int c = cbase + j * 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = ck + g4 + q;
        double v = 0.0;
        if (c < p.N && k < sg.K) v = TRANSB ? B[(int64_t)c * sg.ldb + k] : B[(int64_t)k * sg.ldb + c];
        b[j][q] = (CT)v;
      }
    }
    ck += 16;
    if (ck >= sg.K) {
      cs++;
      ck = 0;
    }
  };
  auto compute = [&](CT (&a)[SM][4], CT (&b)[SN][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          if constexpr (F64)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
        }
  };
  if (nseg > 0) {
    load(a0, b0);
    while (true) {
      const bool h1 = cs < nseg;
      if (h1) load(a1, b1);
      compute(a0, b0);
      if (!h1) break;
      const bool h0 = cs < nseg;
      if (h0) load(a0, b0);
      compute(a1, b1);
      if (!h0) break;
    }
  }
  BST_G TC* __restrict__ C = (BST_G TC*)(ptrs[p.c_buf]) + p.c_off;
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = t.m0 + wm * WM + i * 16 + (F64 ? (4 * r + (lane >> 4)) : (4 * (lane >> 4) + r));
        const int col = t.n0 + wn * WN + j * 16 + r16;
        if (row < p.M && col < p.N) C[(int64_t)row * p.ldc + col] = (TC)acc[i][j][r];
      }
}

// ---------------------------------------------------------------- launchers
template <int FORM, typename TA, typename TC, bool TRANSB>
hipError_t direct_shape(int bm, int bn, const GemmLaunch& g, hipStream_t s) {
  dim3 grid((unsigned)g.ntiles), block(256);
#define BST_DS(BM_, BN_)                                                                             \
  if (bm == BM_ && bn == BN_) {                                                                      \
    hipLaunchKernelGGL((gemm_direct_kernel<FORM, TA, TC, TRANSB, BM_, BN_>), grid, block, 0, s, g.tiles, \
                       g.probs, g.segs, g.ptrs);                                                     \
    return hipGetLastError();                                                                        \
  }
  BST_DS(64, 64) BST_DS(128, 64) BST_DS(64, 128) BST_DS(32, 32)
#undef BST_DS
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_direct(const GemmLaunch& g, int bm, int bn, hipStream_t s) {
  if (g.ntiles <= 0) return hipSuccess;
  const bool a64 = g.ta == ElemType::F64, c64 = g.tc == ElemType::F64;
  if (g.form == BST_FP64) {
    if (!(a64 && c64)) return hipErrorInvalidValue;
    return g.transb ? direct_shape<BST_FP64, double, double, true>(bm, bn, g, s)
                    : direct_shape<BST_FP64, double, double, false>(bm, bn, g, s);
  }
  if (g.form == BST_FP32) {
    if (a64 && c64)
      return g.transb ? direct_shape<BST_FP32, double, double, true>(bm, bn, g, s)
                      : direct_shape<BST_FP32, double, double, false>(bm, bn, g, s);
    if (a64 && !c64 && !g.transb) return direct_shape<BST_FP32, double, float, false>(bm, bn, g, s);
    if (!a64 && c64 && g.transb) return direct_shape<BST_FP32, float, double, true>(bm, bn, g, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace bst

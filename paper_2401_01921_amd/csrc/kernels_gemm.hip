// Grouped sector GEMM for block-sparse contraction on CDNA4 (gfx950) MFMA.
//
// One launch covers every output block ("problem") of a contraction step.
// Each workgroup owns one BM x BN output tile of one problem and sums the
// problem's K-segments (one per matching contracted sector tuple) in a fixed
// order into registers, then writes the tile once: no atomics, so results
// are bitwise reproducible run to run.  Problems without segments produce
// zero tiles (output blocks that no sector pair reaches).
//
// Arithmetic forms (operands arrive as float64 or float32 and are converted
// on the way into LDS, so no separate conversion pass touches HBM):
//   FP64    v_mfma_f64_16x16x4f64,   double accumulate
//   FP32    v_mfma_f32_16x16x4f32,   operands rounded to float32 (RNE)
//   BF16X3  v_mfma_f32_16x16x32_bf16, a = a0 + a1 split, a0b0+a0b1+a1b0
//   BF16X6  same with a2: a0b0+a0b1+a1b0+a0b2+a1b1+a2b0
// Tiles: 4 waves (wave64) in a 2 x 2 arrangement, each wave a
// (BM/2) x (BN/2) patch of 16 x 16 MFMA sub-tiles.
#include "bst_internal.h"

namespace bst {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// Direct (LDS-free) variants first: index 0 is the default.
static const std::vector<TileShape> kShapesF64 = {{64, 64, 1}, {128, 64, 1}, {64, 128, 1}, {32, 32, 1},
                                                  {32, 32, 0}, {64, 64, 0}, {64, 32, 0}, {32, 64, 0}};
static const std::vector<TileShape> kShapesF32 = {{64, 64, 1}, {128, 64, 1}, {64, 128, 1}, {32, 32, 1},
                                                  {32, 32, 0}, {64, 64, 0}, {128, 64, 0}, {64, 128, 0}};
static const std::vector<TileShape> kShapesBF3 = {{32, 32}, {64, 64}, {128, 64}, {64, 128}};
static const std::vector<TileShape> kShapesBF6 = {{32, 32}, {64, 64}};

const std::vector<TileShape>& gemm_tile_shapes(bst_precision form) {
  switch (form) {
    case BST_FP64: return kShapesF64;
    case BST_FP32: return kShapesF32;
    case BST_BF16X3: return kShapesBF3;
    default: return kShapesBF6;
  }
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <int NP>
__device__ __forceinline__ void split_bf16(double a, unsigned short* h) {
  float f = (float)a;
  h[0] = bf16_rne(f);
  if constexpr (NP > 1) {
    double r = a - (double)bf16_val(h[0]);
    h[1] = bf16_rne((float)r);
    if constexpr (NP > 2) {
      double r2 = r - (double)bf16_val(h[1]);
      h[2] = bf16_rne((float)r2);
    }
  }
}
template <int NP>
__device__ __forceinline__ void split_bf16(float a, unsigned short* h) {
  h[0] = bf16_rne(a);
  if constexpr (NP > 1) {
    float r = a - bf16_val(h[0]);  // exact: fewer than 24 significant bits
    h[1] = bf16_rne(r);
    if constexpr (NP > 2) {
      float r2 = r - bf16_val(h[1]);
      h[2] = bf16_rne(r2);
    }
  }
}

template <int FORM> struct FormTraits;
template <> struct FormTraits<BST_FP64> { static constexpr int BK = 16; static constexpr int NP = 0; };
template <> struct FormTraits<BST_FP32> { static constexpr int BK = 16; static constexpr int NP = 0; };
template <> struct FormTraits<BST_BF16X3> { static constexpr int BK = 32; static constexpr int NP = 2; };
template <> struct FormTraits<BST_BF16X6> { static constexpr int BK = 32; static constexpr int NP = 3; };

// Output element (row, col) of lane `lane`, register r of a 16x16 MFMA tile.
// float32 accumulators: row = 4*(lane/16) + r; float64: row = 4*r + lane/16.
template <bool F64ACC>
__device__ __forceinline__ int acc_row(int lane, int r) {
  return F64ACC ? (4 * r + lane / 16) : (4 * (lane / 16) + r);
}

template <int FORM, typename TA, typename TC, bool TRANSB, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(const GemmTile* __restrict__ tiles,
                                                           const GemmProb* __restrict__ probs,
                                                           const GemmSeg* __restrict__ segs,
                                                           void* const* __restrict__ ptrs) {
  constexpr int BK = FormTraits<FORM>::BK;
  constexpr int NP = FormTraits<FORM>::NP;
  constexpr bool F64 = (FORM == BST_FP64);
  constexpr bool BF = (NP > 0);
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int SM = WM / 16, SN = WN / 16;
  using CT = typename std::conditional<F64, double, float>::type;      // MFMA operand (non-bf16)
  using ACC = typename std::conditional<F64, dbl4, flt4>::type;
  constexpr int PADF = 2;   // float/double LDS row pad (elements)
  constexpr int PADH = 8;   // bf16 LDS row pad (elements): keeps 16-byte alignment
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;   // tile elements per thread

  // LDS, double buffered: plain forms store [BK][BM+PADF] (k-major), bf16
  // forms store planes [NP][BM][BK+PADH] (k contiguous, 16-byte lane reads).
  constexpr int A_ELEMS = BF ? NP * BM * (BK + PADH) : BK * (BM + PADF);
  constexpr int B_ELEMS = BF ? NP * BN * (BK + PADH) : BK * (BN + PADF);
  using LT = typename std::conditional<BF, unsigned short, CT>::type;
  __shared__ __attribute__((aligned(16))) LT As[2][A_ELEMS];
  __shared__ __attribute__((aligned(16))) LT Bs[2][B_ELEMS];

  const GemmTile t = tiles[blockIdx.x];
  if (t.prob < 0) return;   // padding of the per-XCD tile lists
  const GemmProb p = probs[t.prob];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = t.m0, n0 = t.n0;

  ACC acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = ACC{0, 0, 0, 0};

  // next k-step to fetch: segment ls, offset lk; values staged in registers
  int ls = 0, lk = 0;
  TA ra[EA];
  double rb[EB];
  auto fetch = [&]() {
    const GemmSeg g = segs[p.seg_begin + ls];
    const BST_G TA* __restrict__ A = (const BST_G TA*)(ptrs[g.a_buf]) + g.a_off;
    const BST_G double* __restrict__ B = (const BST_G double*)(ptrs[g.b_buf]) + g.b_off;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / BK, k = idx % BK;
      const int gr = m0 + r, gk = lk + k;
      ra[e] = (gr < p.M && gk < g.K) ? A[(int64_t)gr * g.lda + gk] : TA(0);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if constexpr (TRANSB) { n = idx / BK; k = idx % BK; }
      else { k = idx / BN; n = idx % BN; }
      const int gn = n0 + n, gk = lk + k;
      double v = 0.0;
      if (gn < p.N && gk < g.K) v = TRANSB ? B[(int64_t)gn * g.ldb + gk] : B[(int64_t)gk * g.ldb + gn];
      rb[e] = v;
    }
    lk += BK;
    if (lk >= g.K) {
      ls++;
      lk = 0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / BK, k = idx % BK;
      if constexpr (BF) {
        unsigned short h[3];
        split_bf16<NP>(ra[e], h);
#pragma unroll
        for (int q = 0; q < NP; ++q) As[buf][(q * BM + r) * (BK + PADH) + k] = h[q];
      } else {
        As[buf][k * (BM + PADF) + r] = (CT)ra[e];
      }
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if constexpr (TRANSB) { n = idx / BK; k = idx % BK; }
      else { k = idx / BN; n = idx % BN; }
      if constexpr (BF) {
        unsigned short h[3];
        split_bf16<NP>(rb[e], h);
#pragma unroll
        for (int q = 0; q < NP; ++q) Bs[buf][(q * BN + n) * (BK + PADH) + k] = h[q];
      } else {
        Bs[buf][k * (BN + PADF) + n] = (CT)rb[e];
      }
    }
  };
  auto compute = [&](int buf) {
    if constexpr (BF) {
      bf16x8 a[NP][SM], b[NP][SN];
      const int kl = 8 * (lane >> 4);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int i = 0; i < SM; ++i) {
          const int r = wm * WM + i * 16 + (lane & 15);
          us8 raw = *reinterpret_cast<const us8*>(&As[buf][(q * BM + r) * (BK + PADH) + kl]);
          a[q][i] = __builtin_bit_cast(bf16x8, raw);
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const int c = wn * WN + j * 16 + (lane & 15);
          us8 raw = *reinterpret_cast<const us8*>(&Bs[buf][(q * BN + c) * (BK + PADH) + kl]);
          b[q][j] = __builtin_bit_cast(bf16x8, raw);
        }
      }
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          if constexpr (NP == 3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int k = kk + (lane >> 4);
        CT a[SM], b[SN];
#pragma unroll
        for (int i = 0; i < SM; ++i) a[i] = As[buf][k * (BM + PADF) + wm * WM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < SN; ++j) b[j] = Bs[buf][k * (BN + PADF) + wn * WN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
          for (int j = 0; j < SN; ++j) {
            if constexpr (F64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
          }
      }
    }
  };

  // pipeline: the next k-step's global loads are in flight while the
  // current one runs on the MFMA units; one barrier per k-step
  if (p.seg_count > 0) {
    fetch();
    stage(0);
    __syncthreads();
    int buf = 0;
    while (true) {
      const bool more = ls < p.seg_count;
      if (more) fetch();
      compute(buf);
      if (more) stage(buf ^ 1);
      __syncthreads();
      buf ^= 1;
      if (!more) break;
    }
  }
  // ---- epilogue: each element written exactly once ----
  BST_G TC* __restrict__ C = (BST_G TC*)(ptrs[p.c_buf]) + p.c_off;
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + acc_row<F64>(lane, r);
        const int col = n0 + wn * WN + j * 16 + (lane & 15);
        if (row < p.M && col < p.N) C[(int64_t)row * p.ldc + col] = (TC)acc[i][j][r];
      }
}

template <int FORM, typename TA, typename TC, bool TRANSB>
static hipError_t launch_shape(int bm, int bn, const GemmLaunch& g, hipStream_t s) {
  dim3 grid((unsigned)g.ntiles), block(256);
#define BST_SHAPE(BM_, BN_)                                                                  \
  if (bm == BM_ && bn == BN_) {                                                              \
    hipLaunchKernelGGL((gemm_grouped_kernel<FORM, TA, TC, TRANSB, BM_, BN_>), grid, block, 0, \
                       s, g.tiles, g.probs, g.segs, g.ptrs);                                 \
    return hipGetLastError();                                                                \
  }
  if constexpr (FORM == BST_FP64) {
    BST_SHAPE(32, 32) BST_SHAPE(64, 64) BST_SHAPE(64, 32) BST_SHAPE(32, 64)
  } else if constexpr (FORM == BST_FP32) {
    BST_SHAPE(32, 32) BST_SHAPE(64, 64) BST_SHAPE(128, 64) BST_SHAPE(64, 128)
  } else {
    BST_SHAPE(32, 32) BST_SHAPE(64, 64)
    if constexpr (FORM == BST_BF16X3) { BST_SHAPE(128, 64) BST_SHAPE(64, 128) }
  }
#undef BST_SHAPE
  return hipErrorInvalidValue;
}

template <int FORM>
static hipError_t launch_form(const GemmLaunch& g, hipStream_t s) {
  const auto& shapes = gemm_tile_shapes((bst_precision)FORM);
  if (g.tile < 0 || g.tile >= (int)shapes.size()) return hipErrorInvalidValue;
  const int bm = shapes[g.tile].bm, bn = shapes[g.tile].bn;
  if (shapes[g.tile].direct) return launch_gemm_direct(g, bm, bn, s);
  const bool a64 = g.ta == ElemType::F64, c64 = g.tc == ElemType::F64;
  if (g.tb != ElemType::F64) return hipErrorInvalidValue;
  if (a64 && c64) {
    return g.transb ? launch_shape<FORM, double, double, true>(bm, bn, g, s)
                    : launch_shape<FORM, double, double, false>(bm, bn, g, s);
  }
  if constexpr (FORM != BST_FP64) {
    if (a64 && !c64 && !g.transb) return launch_shape<FORM, double, float, false>(bm, bn, g, s);
    if (!a64 && c64 && g.transb) return launch_shape<FORM, float, double, true>(bm, bn, g, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm(const GemmLaunch& g, hipStream_t s) {
  if (g.ntiles <= 0) return hipSuccess;
  if (g.ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  switch (g.form) {
    case BST_FP64: return launch_form<BST_FP64>(g, s);
    case BST_FP32: return launch_form<BST_FP32>(g, s);
    case BST_BF16X3: return launch_form<BST_BF16X3>(g, s);
    case BST_BF16X6: return launch_form<BST_BF16X6>(g, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace bst

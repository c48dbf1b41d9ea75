// Split-bfloat16 path: conversion of float64 operands into bfloat16 planes
// (a = a0 + a1 [+ a2], each plane rounded to nearest even) laid out for the
// MFMA loads, and the grouped GEMM that consumes them.
//
// Splitting once per operand instead of once per tile load removes the
// redundant conversions (each element of A is otherwise re-split for every
// N-tile) and halves the bytes the GEMM streams (4 or 6 bytes instead of 8).
// Planes are interleaved by 8-element chunks (plane_at) and operand rows
// padded to 32 elements, so that one 32-deep k step of a row, all planes,
// is one contiguous run of 16-byte vectors (a 128-byte line for two planes).
#include "bst_internal.h"

namespace bst {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short rne_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <int NP>
__device__ __forceinline__ void split_planes(double a, unsigned short* h) {
  h[0] = rne_bf16((float)a);
  double r = a - (double)bf16f(h[0]);
  h[1] = rne_bf16((float)r);
  if constexpr (NP > 2) h[2] = rne_bf16((float)(r - (double)bf16f(h[1])));
}
template <int NP>
__device__ __forceinline__ void split_planes(float a, unsigned short* h) {
  h[0] = rne_bf16(a);
  float r = a - bf16f(h[0]);
  h[1] = rne_bf16(r);
  if constexpr (NP > 2) h[2] = rne_bf16(r - bf16f(h[1]));
}

// ------------------------------------------------------------------------
// float64 blocks -> bfloat16 planes (optionally transposed), 64x64 tiles
// ------------------------------------------------------------------------
template <int NP, typename TI>
__global__ __launch_bounds__(256) void split_kernel(const SplitItem* __restrict__ items,
                                                    void* const* __restrict__ ptrs) {
  // One 64 x 64 tile of the output per workgroup; every lane converts 8
  // consecutive output elements and writes them as one 16-byte vector per
  // plane (output rows are padded to 8, so the vectors are aligned).  A
  // transposed tile is staged in LDS already split: two planes pack into
  // one 32-bit word (half the LDS of a float64 tile, so twice the
  // workgroups per CU), three planes and plain float64 copies stage the
  // input value.
  using TS = typename std::conditional<NP == 2, uint32_t, TI>::type;
  __shared__ TS tile[64][65];
  const SplitItem j = items[blockIdx.x];
  const BST_G TI* __restrict__ in = (const BST_G TI*)(ptrs[j.in_buf]) + j.in_off;
  BST_G unsigned short* __restrict__ out = (BST_G unsigned short*)(ptrs[j.out_buf]);
  const int tid = threadIdx.x;
  const int orow = tid >> 3, ocol = (tid & 7) * 8;   // 32 rows x 8 vectors per pass
  if (!j.transpose) {
    // output [rows x out_ld]: rows r0.., columns c0.. (zeros past cols)
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int r = j.r0 + orow + 32 * pass, c = j.c0 + ocol;
      if (r < j.rows && c < j.out_ld) {
        if constexpr (NP == 1) {   // float64 copy into the padded layout
          dbl4 v[2];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e >> 2][e & 3] = (c + e) < j.cols ? (double)in[(int64_t)r * j.cols + c + e] : 0.0;
          BST_G dbl4* o = (BST_G dbl4*)((BST_G double*)(ptrs[j.out_buf]) + j.out_off + (int64_t)r * j.out_ld + c);
          o[0] = v[0];
          o[1] = v[1];
          continue;
        }
        us8 h[3];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double v = (c + e) < j.cols ? (double)in[(int64_t)r * j.cols + c + e] : 0.0;
          unsigned short t[3];
          split_planes<NP>(v, t);
#pragma unroll
          for (int q = 0; q < NP; ++q) h[q][e] = t[q];
        }
        const int64_t pos = j.out_off + (int64_t)r * j.out_ld + c;   // a multiple of 8
#pragma unroll
        for (int q = 0; q < NP; ++q) *reinterpret_cast<BST_G us8*>(out + plane_at(NP, pos, q)) = h[q];
      }
    }
    return;
  }
  // transposed: input [rows x cols] -> output [cols x out_ld], out_ld >= rows;
  // all sixteen loads of a lane in flight before the first LDS store
  TI v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = tid + 256 * i;
    const int gr = j.r0 + (e >> 6), gc = j.c0 + (e & 63);
    v[i] = (gr < j.rows && gc < j.cols) ? in[(int64_t)gr * j.cols + gc] : (TI)0;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = tid + 256 * i;
    if constexpr (NP == 2) {
      unsigned short t[3];
      split_planes<2>(v[i], t);
      tile[e >> 6][e & 63] = (uint32_t)t[0] | ((uint32_t)t[1] << 16);
    } else {
      tile[e >> 6][e & 63] = v[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int c = orow + 32 * pass;          // output row = input column
    const int gc = j.c0 + c, gr = j.r0 + ocol;
    if (gc < j.cols && gr < j.out_ld) {
      if constexpr (NP == 1) {
        dbl4 o8[2];
#pragma unroll
        for (int e = 0; e < 8; ++e) o8[e >> 2][e & 3] = (double)tile[ocol + e][c];
        BST_G dbl4* o = (BST_G dbl4*)((BST_G double*)(ptrs[j.out_buf]) + j.out_off + (int64_t)gc * j.out_ld + gr);
        o[0] = o8[0];
        o[1] = o8[1];
        continue;
      }
      us8 h[3];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (NP == 2) {
          const uint32_t u = tile[ocol + e][c];
          h[0][e] = (unsigned short)(u & 0xFFFFu);
          h[1][e] = (unsigned short)(u >> 16);
        } else {
          unsigned short t[3];
          split_planes<NP>(tile[ocol + e][c], t);
#pragma unroll
          for (int q = 0; q < NP; ++q) h[q][e] = t[q];
        }
      }
      const int64_t pos = j.out_off + (int64_t)gc * j.out_ld + gr;   // a multiple of 8
#pragma unroll
      for (int q = 0; q < NP; ++q) *reinterpret_cast<BST_G us8*>(out + plane_at(NP, pos, q)) = h[q];
    }
  }
}

hipError_t launch_split(const SplitLaunch& l, hipStream_t s) {
  if (l.nwork <= 0) return hipSuccess;
  if (l.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)l.nwork), block(256);
  if (l.np == 1 && !l.in_f32)
    hipLaunchKernelGGL((split_kernel<1, double>), grid, block, 0, s, l.items, l.ptrs);
  else if (l.np == 2 && !l.in_f32)
    hipLaunchKernelGGL((split_kernel<2, double>), grid, block, 0, s, l.items, l.ptrs);
  else if (l.np == 2)
    hipLaunchKernelGGL((split_kernel<2, float>), grid, block, 0, s, l.items, l.ptrs);
  else if (l.np == 3 && !l.in_f32)
    hipLaunchKernelGGL((split_kernel<3, double>), grid, block, 0, s, l.items, l.ptrs);
  else if (l.np == 3)
    hipLaunchKernelGGL((split_kernel<3, float>), grid, block, 0, s, l.items, l.ptrs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// Grouped GEMM on bfloat16 planes: C[M x N] = sum_seg A[M x K] B[N x K]^T
// ------------------------------------------------------------------------
// An LDS operand row holds one 32-deep k step of all NP planes: NC = 4 * NP
// 16-byte pieces, piece cc = chunk * NP + plane, in the order of the
// interleaved global layout.  Piece cc of row r sits at position swz(r, cc),
// an involution for a fixed r that spreads the 16 rows one MFMA operand
// read touches (same cc) over distinct bank groups; a row's pieces are
// stored by consecutive lanes.
template <int NP>
__device__ __forceinline__ int swz(int r, int cc) {
  if constexpr (NP == 2) return cc ^ ((r >> 1) & 7);
  return (cc & ~3) | ((cc ^ (r >> 1)) & 3);
}

// Tile shapes per plane count: the LDS-staged kernel (index 0, 64x64, is
// the default) and the pipelined kernel (kind 3, kernels_stream.hip).
static const std::vector<TileShape> kPlaneShapes2 = {
    {64, 64, 0},         {128, 64, 0},        {64, 128, 0},       {32, 32, 0},     {128, 128, 0},
    {128, 64, 3, 3, 4},  {64, 128, 3, 3, 4},  {128, 128, 3, 3, 8}, {128, 256, 3, 3, 8},
    {256, 128, 3, 3, 8}, {256, 64, 3, 3, 8},  {64, 192, 3, 3, 4}, {64, 192, 3, 2, 4},
    {128, 192, 3, 3, 8}, {128, 128, 3, 2, 8}, {128, 64, 3, 2, 4}, {64, 128, 3, 2, 4},
    {32, 192, 3, 2, 4}};
static const std::vector<TileShape> kPlaneShapes3 = {{64, 64, 0}, {32, 32, 0}, {64, 64, 3, 3, 4},
                                                     {128, 128, 3, 3, 8}};
// float64 operands in the padded layouts: the pipelined kernel only
static const std::vector<TileShape> kPlaneShapes1 = {{64, 64, 3, 3, 4},   {128, 64, 3, 3, 4},
                                                     {64, 128, 3, 3, 4},  {128, 128, 3, 3, 8},
                                                     {256, 128, 3, 3, 8}, {128, 256, 3, 3, 8},
                                                     {64, 64, 3, 2, 4},   {128, 64, 3, 2, 4},
                                                     {64, 128, 3, 2, 4},  {128, 128, 3, 2, 8}};
const std::vector<TileShape>& gemm_planes_shapes(int np) {
  return np == 1 ? kPlaneShapes1 : np == 3 ? kPlaneShapes3 : kPlaneShapes2;
}

template <int NP, typename TC, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void gemm_planes_kernel(const GemmTile* __restrict__ tiles,
                                                          const GemmProb* __restrict__ probs,
                                                          const GemmSeg* __restrict__ segs,
                                                          void* const* __restrict__ ptrs,
                                                          const int64_t* __restrict__ rowmap) {
  // LDS row: one BK-deep k step (64 or 128 bytes), 16-byte chunks swizzled
  constexpr int CH = BK / 8, NC = NP * CH;   // 16-byte pieces per row and k step
  constexpr int WM = BM / 2, WN = BN / 2, SM = WM / 16, SN = WN / 16;
  constexpr int NVA = (BM * NC + 255) / 256, NVB = (BN * NC + 255) / 256;   // pieces per thread
  static_assert(BK == 32, "one 32-deep k step per LDS row");
  __shared__ __attribute__((aligned(16))) unsigned short As[2][BM * NC * 8];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][BN * NC * 8];

  const GemmTile t = tiles[blockIdx.x];
  if (t.prob < 0) return;   // padding of the per-XCD tile lists
  const GemmProb p = probs[t.prob];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = t.m0, n0 = t.n0;

  flt4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = flt4{0, 0, 0, 0};

  // Loads only issue the 16-byte reads; rows past M / N and k past the
  // segment's K are zeroed when the registers go to LDS (after the MFMAs),
  // so no wait for the data sits between the loads.  Piece e of a row's
  // k step is chunk e / NP of plane e % NP: consecutive lanes read one
  // contiguous run (plane_at), NC pieces per row.
  us8 ra[NVA], rb[NVB];
  int na[NVA], nb[NVB];   // valid k elements of each piece (0..8)

  // cursor of the next k-step to load: segment ls (cached), offset lk
  int ls = 0, lk = 0;
  GemmSeg lg{};
  const BST_G unsigned short* lA = nullptr;
  const BST_G unsigned short* lB = nullptr;
  auto set_seg = [&]() {
    lg = segs[p.seg_begin + ls];
    lA = (const BST_G unsigned short*)(ptrs[lg.a_buf]);
    lB = (const BST_G unsigned short*)(ptrs[lg.b_buf]);
  };
  auto load = [&]() {
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      const int r = idx / NC, e = idx % NC;
      const int kv = lk + (e / NP) * 8;
      const int gr = m0 + r;
      const bool ok = (idx < BM * NC) && gr < p.M && kv < lg.K;
      na[v] = ok ? min(8, lg.K - kv) : 0;
      if (ok)
        ra[v] = *reinterpret_cast<const BST_G us8*>(
            lA + plane_at(NP, lg.a_off + (int64_t)gr * lg.lda + kv, e % NP));
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      const int r = idx / NC, e = idx % NC;
      const int kv = lk + (e / NP) * 8;
      const int gn = n0 + r;
      const bool ok = (idx < BN * NC) && gn < p.N && kv < lg.K;
      nb[v] = ok ? min(8, lg.K - kv) : 0;
      if (ok)
        rb[v] = *reinterpret_cast<const BST_G us8*>(
            lB + plane_at(NP, lg.b_off + (int64_t)gn * lg.ldb + kv, e % NP));
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      if (idx < BM * NC) {
        const int r = idx / NC, e = idx % NC;
        us8 x = ra[v];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k >= na[v]) x[k] = 0;
        *reinterpret_cast<us8*>(&As[buf][r * NC * 8 + swz<NP>(r, e) * 8]) = x;
      }
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      if (idx < BN * NC) {
        const int r = idx / NC, e = idx % NC;
        us8 x = rb[v];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k >= nb[v]) x[k] = 0;
        *reinterpret_cast<us8*>(&Bs[buf][r * NC * 8 + swz<NP>(r, e) * 8]) = x;
      }
    }
  };
  auto advance = [&]() {
    lk += BK;
    if (lk >= lg.K) {
      ls++;
      lk = 0;
      if (ls < p.seg_count) set_seg();
    }
  };

  int buf = 0;
  if (p.seg_count > 0) {
    set_seg();
    load();
    advance();
    store(0);
  }
  __syncthreads();
  bool more = p.seg_count > 0;
  while (more) {
    const bool have_next = ls < p.seg_count;
    if (have_next) load();
    // MFMA on the current buffer, BK / 32 steps of 32
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      const int kc = (lane >> 4) + 4 * ks;   // 8-element k chunk of this lane
      bf16x8 a[NP][SM], b[NP][SN];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int i = 0; i < SM; ++i) {
          const int r = wm * WM + i * 16 + (lane & 15);
          a[q][i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&As[buf][r * NC * 8 + swz<NP>(r, kc * NP + q) * 8]));
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const int c = wn * WN + j * 16 + (lane & 15);
          b[q][j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Bs[buf][c * NC * 8 + swz<NP>(c, kc * NP + q) * 8]));
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
    }
    if (have_next) {
      advance();
      store(buf ^ 1);
    }
    __syncthreads();
    buf ^= 1;
    more = have_next;
  }
  BST_G TC* __restrict__ C = (BST_G TC*)(ptrs[p.c_buf]);
  // all row offsets first (row-mapped problems read them from the table)
  int64_t rbase[SM][4];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm * WM + i * 16 + 4 * (lane >> 4) + r;
      rbase[i][r] = row >= p.M ? -1
                               : (p.rowmap1 > 0 ? rowmap[p.rowmap1 - 1 + row] : p.c_off + (int64_t)row * p.ldc);
    }
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (rbase[i][r] < 0) continue;
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        const int col = n0 + wn * WN + j * 16 + (lane & 15);
        if (col < p.N) C[rbase[i][r] + col] = (TC)acc[i][j][r];
      }
    }
}

template <int NP, typename TC>
static hipError_t planes_shape(int bm, int bn, int bk, const PlanesLaunch& g, hipStream_t s) {
  dim3 grid((unsigned)g.ntiles), block(256);
#define BST_PS(BM_, BN_, BK_)                                                                   \
  if (bm == BM_ && bn == BN_ && bk == BK_) {                                                    \
    hipLaunchKernelGGL((gemm_planes_kernel<NP, TC, BM_, BN_, BK_>), grid, block, 0, s, g.tiles,  \
                       g.probs, g.segs, g.ptrs, g.rowmap);                                      \
    return hipGetLastError();                                                                   \
  }
  BST_PS(64, 64, 32) BST_PS(32, 32, 32)
  if constexpr (NP == 2) {
    BST_PS(128, 64, 32) BST_PS(64, 128, 32) BST_PS(128, 128, 32)
  }
#undef BST_PS
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_planes(const PlanesLaunch& g, hipStream_t s) {
  if (g.ntiles <= 0) return hipSuccess;
  if (g.ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  const auto& sh = gemm_planes_shapes(g.np);
  if (g.tile < 0 || g.tile >= (int)sh.size()) return hipErrorInvalidValue;
  const int bm = sh[g.tile].bm, bn = sh[g.tile].bn;
  if (sh[g.tile].direct != 0) return hipErrorInvalidValue;   // kind 3: launch_gemm_planes_stream
  const int bk = 32;   // 64-deep k steps (1 or 2 workgroups per CU) measured slower
  if (g.np == 2)
    return g.tc == ElemType::F64 ? planes_shape<2, double>(bm, bn, bk, g, s)
                                 : planes_shape<2, float>(bm, bn, bk, g, s);
  if (g.np == 3)
    return g.tc == ElemType::F64 ? planes_shape<3, double>(bm, bn, bk, g, s)
                                 : planes_shape<3, float>(bm, bn, bk, g, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------
// Two-site MPO apply writing its output as bfloat16 planes
// ------------------------------------------------------------------------
template <int NMAX, int NP>
__global__ __launch_bounds__(256) void happly_planes_kernel(const HTask* __restrict__ tasks,
                                                            const HPlane* __restrict__ planes,
                                                            const HWork* __restrict__ work,
                                                            void* const* __restrict__ ptrs,
                                                            const float* __restrict__ coef) {
  __shared__ float cf[NMAX * NMAX];
  __shared__ HPlane pl[2 * NMAX];
  const HWork w = work[blockIdx.x];
  const HTask t = tasks[w.task];
  const int tid = threadIdx.x;
  for (int e = tid; e < NMAX * NMAX; e += 256) cf[e] = coef[(int64_t)t.cls * NMAX * NMAX + e];
  for (int e = tid; e < t.nin + t.nout; e += 256) pl[e] = planes[t.plane_begin + e];
  __syncthreads();
  const int site = w.site0 + tid;
  if (site >= t.rows * t.cols) return;
  const int i = site / t.cols, jc = site % t.cols;
  const BST_G float* __restrict__ in = (const BST_G float*)(ptrs[t.in_buf]);
  BST_G unsigned short* __restrict__ out = (BST_G unsigned short*)(ptrs[t.out_buf]);
  float x[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k)
    x[k] = (k < t.nin) ? in[pl[k].off + (int64_t)i * pl[k].rowstride + jc] : 0.0f;
#pragma unroll
  for (int o = 0; o < NMAX; ++o) {
    if (o < t.nout) {
      float y = 0.0f;
#pragma unroll
      for (int k = 0; k < NMAX; ++k) y += cf[o * NMAX + k] * x[k];
      const HPlane q = pl[t.nin + o];
      unsigned short h[3];
      split_planes<NP>(y, h);
      const int64_t at = q.off + (int64_t)i * q.rowstride + jc;
#pragma unroll
      for (int pq = 0; pq < NP; ++pq) out[plane_at(NP, at, pq)] = h[pq];
    }
  }
}

hipError_t launch_happly_planes(const HApplyLaunch& h, hipStream_t s) {
  if (h.nwork <= 0) return hipSuccess;
  if (h.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  dim3 grid((unsigned)h.nwork), block(256);
  const float* cf = reinterpret_cast<const float*>(h.coef);
#define BST_HP(N_, P_)                                                                            \
  if (h.nmax == N_ && h.np == P_) {                                                               \
    hipLaunchKernelGGL((happly_planes_kernel<N_, P_>), grid, block, 0, s, h.tasks, h.planes, h.work, \
                       h.ptrs, cf);                                                               \
    return hipGetLastError();                                                                     \
  }
  BST_HP(8, 2) BST_HP(16, 2) BST_HP(32, 2) BST_HP(64, 2)
  BST_HP(8, 3) BST_HP(16, 3) BST_HP(32, 3) BST_HP(64, 3)
#undef BST_HP
  return hipErrorInvalidValue;
}

}  // namespace bst

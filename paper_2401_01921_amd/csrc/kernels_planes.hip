// Split-bfloat16 path: conversion of float64 operands into bfloat16 planes
// (a = a0 + a1 [+ a2], each plane rounded to nearest even) laid out for the
// MFMA loads, and the grouped GEMM that consumes them.
//
// Splitting once per operand instead of once per tile load removes the
// redundant conversions (each element of A is otherwise re-split for every
// N-tile) and halves the bytes the GEMM streams (4 or 6 bytes instead of 8).
// Plane rows are padded to 8 elements so that every tile row is a whole
// number of 16-byte vectors.
#include "bst_internal.h"

namespace bst {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

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
template <int NP>
__global__ __launch_bounds__(256) void split_kernel(const SplitJob* __restrict__ jobs,
                                                    const SplitWork* __restrict__ work,
                                                    void* const* __restrict__ ptrs) {
  // One 64 x 64 tile of the output per workgroup; every lane converts 8
  // consecutive output elements and writes them as one 16-byte vector per
  // plane (output rows are padded to 8, so the vectors are aligned).
  __shared__ double tile[64][65];
  const SplitWork w = work[blockIdx.x];
  const SplitJob j = jobs[w.job];
  const BST_G double* __restrict__ in = (const BST_G double*)(ptrs[j.in_buf]) + j.in_off;
  BST_G unsigned short* __restrict__ out = (BST_G unsigned short*)(ptrs[j.out_buf]) + j.out_off;
  const int tid = threadIdx.x;
  const int orow = tid >> 3, ocol = (tid & 7) * 8;   // 32 rows x 8 vectors per pass
  if (!j.transpose) {
    // output [rows x out_ld]: rows r0.., columns c0.. (zeros past cols)
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int r = w.r0 + orow + 32 * pass, c = w.c0 + ocol;
      if (r < j.rows && c < j.out_ld) {
        us8 h[3];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double v = (c + e) < j.cols ? in[(int64_t)r * j.cols + c + e] : 0.0;
          unsigned short t[3];
          split_planes<NP>(v, t);
#pragma unroll
          for (int q = 0; q < NP; ++q) h[q][e] = t[q];
        }
#pragma unroll
        for (int q = 0; q < NP; ++q)
          *reinterpret_cast<BST_G us8*>(out + q * j.out_ps + (int64_t)r * j.out_ld + c) = h[q];
      }
    }
    return;
  }
  // transposed: input [rows x cols] -> output [cols x out_ld], out_ld >= rows
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    const int gr = w.r0 + r, gc = w.c0 + c;
    tile[r][c] = (gr < j.rows && gc < j.cols) ? in[(int64_t)gr * j.cols + gc] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int c = orow + 32 * pass;          // output row = input column
    const int gc = w.c0 + c, gr = w.r0 + ocol;
    if (gc < j.cols && gr < j.out_ld) {
      us8 h[3];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        unsigned short t[3];
        split_planes<NP>(tile[ocol + e][c], t);
#pragma unroll
        for (int q = 0; q < NP; ++q) h[q][e] = t[q];
      }
#pragma unroll
      for (int q = 0; q < NP; ++q)
        *reinterpret_cast<BST_G us8*>(out + q * j.out_ps + (int64_t)gc * j.out_ld + gr) = h[q];
    }
  }
}

hipError_t launch_split(const SplitLaunch& l, hipStream_t s) {
  if (l.nwork <= 0) return hipSuccess;
  if (l.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (l.np == 2)
    hipLaunchKernelGGL(split_kernel<2>, dim3((unsigned)l.nwork), dim3(256), 0, s, l.jobs, l.work, l.ptrs);
  else if (l.np == 3)
    hipLaunchKernelGGL(split_kernel<3>, dim3((unsigned)l.nwork), dim3(256), 0, s, l.jobs, l.work, l.ptrs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// Grouped GEMM on bfloat16 planes: C[M x N] = sum_seg A[M x K] B[N x K]^T
// ------------------------------------------------------------------------
// LDS tile rows hold one 32-deep k step: 64 bytes, four 16-byte chunks.
// Chunk c of row r is stored at chunk c ^ ((r >> 2) & 3), so that the 16
// rows one MFMA operand read touches (same chunk) and the 4 rows x 4 chunks
// one 16-lane group stores fall on 16 distinct 4-bank groups.
__device__ __forceinline__ int lds_chunk(int r, int c) { return r * 32 + ((c ^ ((r >> 2) & 3)) << 3); }
// The same for rows of CH chunks (CH = 4: lds_chunk; CH = 8: 128-byte rows,
// chunk c of row r at c ^ ((r >> 1) & 7), again conflict-free for 16 rows of
// one chunk and for the 2 rows x 8 chunks of a 16-lane store).
template <int CH>
__device__ __forceinline__ int lds_at(int r, int c) {
  if constexpr (CH == 4) return lds_chunk(r, c);
  return r * 64 + ((c ^ ((r >> 1) & 7)) << 3);
}

// Tile shapes per plane count (double-buffered LDS: 80 KB at 128x128, two planes).
// Direct (LDS-free) variants first: index 0 is the default.
static const std::vector<TileShape> kPlaneShapes2 = {{64, 64, 1}, {128, 64, 1}, {64, 128, 1}, {32, 32, 1},
                                                     {64, 64, 0}, {128, 64, 0}, {64, 128, 0}, {32, 32, 0},
                                                     {128, 128, 0}, {128, 128, 2}, {64, 64, 2}};
static const std::vector<TileShape> kPlaneShapes3 = {{64, 64, 1}, {128, 64, 1}, {64, 128, 1}, {32, 32, 1},
                                                     {64, 64, 0}, {32, 32, 0}, {64, 64, 2}};
const std::vector<TileShape>& gemm_planes_shapes(int np) { return np == 3 ? kPlaneShapes3 : kPlaneShapes2; }

template <int NP, typename TC, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void gemm_planes_kernel(const GemmTile* __restrict__ tiles,
                                                          const GemmProb* __restrict__ probs,
                                                          const GemmSeg* __restrict__ segs,
                                                          void* const* __restrict__ ptrs,
                                                          const int64_t* __restrict__ rowmap) {
  // LDS row: one BK-deep k step (64 or 128 bytes), 16-byte chunks swizzled
  constexpr int LDR = BK, CH = BK / 8;
  constexpr int WM = BM / 2, WN = BN / 2, SM = WM / 16, SN = WN / 16;
  constexpr int NVA = (BM * CH + 255) / 256, NVB = (BN * CH + 255) / 256;   // 16-byte vectors per thread
  __shared__ __attribute__((aligned(16))) unsigned short As[2][NP][BM * LDR];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NP][BN * LDR];

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
  // so no wait for the data sits between the loads.
  us8 ra[NP][NVA], rb[NP][NVB];
  int na[NVA], nb[NVB];   // valid k elements of each vector (0..8)

  // cursor of the next k-step to load: segment ls (cached), offset lk
  int ls = 0, lk = 0;
  GemmSeg lg{};
  const BST_G unsigned short* lA = nullptr;
  const BST_G unsigned short* lB = nullptr;
  auto set_seg = [&]() {
    lg = segs[p.seg_begin + ls];
    lA = (const BST_G unsigned short*)(ptrs[lg.a_buf]) + lg.a_off;
    lB = (const BST_G unsigned short*)(ptrs[lg.b_buf]) + lg.b_off;
  };
  auto load = [&]() {
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      const int r = idx / CH, kv = lk + (idx % CH) * 8;
      const int gr = m0 + r;
      const bool ok = (idx < BM * CH) && gr < p.M && kv < lg.K;
      na[v] = ok ? min(8, lg.K - kv) : 0;
      if (ok) {
#pragma unroll
        for (int q = 0; q < NP; ++q)
          ra[q][v] = *reinterpret_cast<const BST_G us8*>(lA + q * lg.a_ps + (int64_t)gr * lg.lda + kv);
      }
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      const int r = idx / CH, kv = lk + (idx % CH) * 8;
      const int gn = n0 + r;
      const bool ok = (idx < BN * CH) && gn < p.N && kv < lg.K;
      nb[v] = ok ? min(8, lg.K - kv) : 0;
      if (ok) {
#pragma unroll
        for (int q = 0; q < NP; ++q)
          rb[q][v] = *reinterpret_cast<const BST_G us8*>(lB + q * lg.b_ps + (int64_t)gn * lg.ldb + kv);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      if (idx < BM * CH) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          us8 x = ra[q][v];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (e >= na[v]) x[e] = 0;
          *reinterpret_cast<us8*>(&As[buf][q][lds_at<CH>(idx / CH, idx % CH)]) = x;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      if (idx < BN * CH) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          us8 x = rb[q][v];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (e >= nb[v]) x[e] = 0;
          *reinterpret_cast<us8*>(&Bs[buf][q][lds_at<CH>(idx / CH, idx % CH)]) = x;
        }
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
          a[q][i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&As[buf][q][lds_at<CH>(r, kc)]));
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const int c = wn * WN + j * 16 + (lane & 15);
          b[q][j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Bs[buf][q][lds_at<CH>(c, kc)]));
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

// Persistent variant: a fixed grid (a multiple of 8, so that block b stays
// on XCD b % 8 with the tiles the host placed there) walks the tile list
// with stride gridDim.x.  The load cursor runs one k-step ahead of the MFMA
// across tile boundaries, so the first k-step of the next tile is in flight
// while the current tile finishes and writes its result.
template <int NP, typename TC, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_planes_persist_kernel(
    const GemmTile* __restrict__ tiles, int64_t ntiles, const GemmProb* __restrict__ probs,
    const GemmSeg* __restrict__ segs, void* const* __restrict__ ptrs,
    const int64_t* __restrict__ rowmap) {
  constexpr int BK = 32, LDR = BK;
  constexpr int WM = BM / 2, WN = BN / 2, SM = WM / 16, SN = WN / 16;
  constexpr int NVA = (BM * 4 + 255) / 256, NVB = (BN * 4 + 255) / 256;
  __shared__ __attribute__((aligned(16))) unsigned short As[2][NP][BM * LDR];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NP][BN * LDR];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t G = gridDim.x;
  const us8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};

  auto row_base = [&](const GemmProb& p, int row) -> int64_t {
    return p.rowmap1 > 0 ? rowmap[p.rowmap1 - 1 + row] : p.c_off + (int64_t)row * p.ldc;
  };
  // load cursor: tile index, its problem and origin, segment and k
  int64_t lt = (int64_t)blockIdx.x - G;
  GemmProb lp{};
  int lm0 = 0, ln0 = 0, ls = 0, lk = 0;
  bool lvalid = false;
  // moves the load cursor to the next tile with work; tiles of problems
  // without segments are written as zeros on the way
  auto next_tile = [&]() {
    lvalid = false;
    for (lt += G; lt < ntiles; lt += G) {
      const GemmTile t = tiles[lt];
      if (t.prob < 0) continue;
      lp = probs[t.prob];
      lm0 = t.m0;
      ln0 = t.n0;
      ls = 0;
      lk = 0;
      if (lp.seg_count > 0) {
        lvalid = true;
        return;
      }
      BST_G TC* __restrict__ C = (BST_G TC*)(ptrs[lp.c_buf]);
      for (int e = tid; e < BM * BN; e += 256) {
        const int row = lm0 + e / BN, col = ln0 + e % BN;
        if (row < lp.M && col < lp.N) C[row_base(lp, row) + col] = (TC)0;
      }
    }
  };
  us8 ra[NP][NVA], rb[NP][NVB];
  auto load = [&]() {
    const GemmSeg g = segs[lp.seg_begin + ls];
    const BST_G unsigned short* A = (const BST_G unsigned short*)(ptrs[g.a_buf]) + g.a_off;
    const BST_G unsigned short* B = (const BST_G unsigned short*)(ptrs[g.b_buf]) + g.b_off;
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      const int r = idx >> 2, kv = lk + (idx & 3) * 8;
      const int gr = lm0 + r;
      const bool ok = (idx < BM * 4) && gr < lp.M && kv < g.K;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        us8 x = ok ? *reinterpret_cast<const BST_G us8*>(A + q * g.a_ps + (int64_t)gr * g.lda + kv) : zero8;
        if (ok && kv + 8 > g.K) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (kv + e >= g.K) x[e] = 0;
        }
        ra[q][v] = x;
      }
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      const int r = idx >> 2, kv = lk + (idx & 3) * 8;
      const int gn = ln0 + r;
      const bool ok = (idx < BN * 4) && gn < lp.N && kv < g.K;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        us8 x = ok ? *reinterpret_cast<const BST_G us8*>(B + q * g.b_ps + (int64_t)gn * g.ldb + kv) : zero8;
        if (ok && kv + 8 > g.K) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (kv + e >= g.K) x[e] = 0;
        }
        rb[q][v] = x;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      if (idx < BM * 4) {
#pragma unroll
        for (int q = 0; q < NP; ++q)
          *reinterpret_cast<us8*>(&As[buf][q][lds_chunk(idx >> 2, idx & 3)]) = ra[q][v];
      }
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      if (idx < BN * 4) {
#pragma unroll
        for (int q = 0; q < NP; ++q)
          *reinterpret_cast<us8*>(&Bs[buf][q][lds_chunk(idx >> 2, idx & 3)]) = rb[q][v];
      }
    }
  };
  // true when the cursor's k-step is the last one of its tile
  auto last_step = [&]() -> bool {
    return ls == lp.seg_count - 1 && lk + BK >= segs[lp.seg_begin + ls].K;
  };
  auto advance = [&]() {
    lk += BK;
    if (lk >= segs[lp.seg_begin + ls].K) {
      ++ls;
      lk = 0;
      if (ls >= lp.seg_count) next_tile();
    }
  };

  next_tile();
  if (!lvalid) return;
  flt4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = flt4{0, 0, 0, 0};
  // the tile whose k-step sits in the current buffer
  GemmProb cp = lp;
  int cm0 = lm0, cn0 = ln0;
  bool clast = last_step();
  load();
  advance();
  store(0);
  __syncthreads();
  int buf = 0;
  for (;;) {
    const bool nvalid = lvalid;
    GemmProb np_ = lp;
    int nm0 = lm0, nn0 = ln0;
    bool nlast = false;
    if (nvalid) {
      nlast = last_step();
      load();
      advance();
    }
    {
      const int kc = lane >> 4;   // 8-element k chunk of this lane
      bf16x8 a[NP][SM], b[NP][SN];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int i = 0; i < SM; ++i) {
          const int r = wm * WM + i * 16 + (lane & 15);
          a[q][i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&As[buf][q][lds_chunk(r, kc)]));
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const int c = wn * WN + j * 16 + (lane & 15);
          b[q][j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Bs[buf][q][lds_chunk(c, kc)]));
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
    if (clast) {
      BST_G TC* __restrict__ C = (BST_G TC*)(ptrs[cp.c_buf]);
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = cm0 + wm * WM + i * 16 + 4 * (lane >> 4) + r;
          if (row >= cp.M) continue;
          const int64_t rbase = row_base(cp, row);
#pragma unroll
          for (int j = 0; j < SN; ++j) {
            const int col = cn0 + wn * WN + j * 16 + (lane & 15);
            if (col < cp.N) C[rbase + col] = (TC)acc[i][j][r];
          }
        }
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) acc[i][j] = flt4{0, 0, 0, 0};
    }
    if (!nvalid) break;
    store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    cp = np_;
    cm0 = nm0;
    cn0 = nn0;
    clast = nlast;
  }
}

template <int NP, typename TC>
static hipError_t planes_persist_shape(int bm, int bn, const PlanesLaunch& g, hipStream_t s) {
  // two resident workgroups per CU at 128x128 (80 KB of LDS), four below
  const int per_cu = (bm * bn >= 128 * 128) ? 2 : 4;
  int64_t grid = (int64_t)256 * per_cu;
  if (grid > g.ntiles) grid = (g.ntiles + 7) / 8 * 8;
  dim3 gr((unsigned)grid), block(256);
#define BST_PP(BM_, BN_)                                                                           \
  if (bm == BM_ && bn == BN_) {                                                                    \
    hipLaunchKernelGGL((gemm_planes_persist_kernel<NP, TC, BM_, BN_>), gr, block, 0, s, g.tiles,    \
                       g.ntiles, g.probs, g.segs, g.ptrs, g.rowmap);                               \
    return hipGetLastError();                                                                      \
  }
  BST_PP(64, 64)
  if constexpr (NP == 2) {
    BST_PP(128, 128)
  }
#undef BST_PP
  return hipErrorInvalidValue;
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
  if (sh[g.tile].direct == 1) return launch_gemm_direct_planes(g, bm, bn, s);
  if (sh[g.tile].direct == 2) {
    if (g.np == 2)
      return g.tc == ElemType::F64 ? planes_persist_shape<2, double>(bm, bn, g, s)
                                   : planes_persist_shape<2, float>(bm, bn, g, s);
    return g.tc == ElemType::F64 ? planes_persist_shape<3, double>(bm, bn, g, s)
                                 : planes_persist_shape<3, float>(bm, bn, g, s);
  }
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
      for (int pq = 0; pq < NP; ++pq) out[pq * t.out_ps + at] = h[pq];
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

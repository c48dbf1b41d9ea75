// Pipelined persistent GEMM on bfloat16 planes.
//
// The plane GEMMs of the two-site H_eff apply have short K (one charge
// sector, or a few of them) and many output tiles, so a kernel that loads one
// k-step ahead spends most of its time waiting: on the chain of table reads
// that starts each tile, on the first operand load, and on one memory
// latency per k-step.  This kernel removes the waits instead of hiding them
// behind occupancy:
//   - a fixed grid; every workgroup walks a host-built list of k-steps (one
//     48-byte record each, the steps of a tile consecutive), so no table is
//     read on the critical path;
//   - operand tiles go from global memory straight into LDS
//     (global_load_lds_dwordx4: no registers, no LDS store instructions),
//     S - 1 k-steps ahead of the MFMAs, into a ring of S stages, across tile
//     boundaries, so the first loads of the next tile are in flight while the
//     current one finishes and writes its result;
//   - the step records themselves are copied into LDS 16 at a time, one batch
//     ahead; the row offsets of row-mapped tiles are copied at the tile's
//     first step.
// Waits are explicit: before k-step u the wave waits until only the copies
// issued after step u's copies are outstanding (vector memory operations
// complete in issue order on this target) and then meets the other waves at
// a barrier.  Copies that are not counted (record batches, row offsets)
// only make a wait stricter.  The stores of a tile are counted exactly: every
// lane stores every element, lanes outside the tile to a sink.
#include "bst_internal.h"

#pragma clang diagnostic ignored "-Winline-asm"

namespace bst {

namespace {
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef double dbl4 __attribute__((ext_vector_type(4)));
#define BST_LDS __attribute__((address_space(3)))

// An LDS operand row holds one 32-deep k step of all NP planes: NC = 4 * NP
// 16-byte pieces, piece cc = chunk * NP + plane, in global order (so that
// the lanes copying a row read one contiguous run).  Piece cc of row r sits
// at position swz(r, cc), an involution for a fixed r that spreads the 16
// rows one MFMA operand read touches (same cc) over distinct bank groups.
template <int NP>
__device__ __forceinline__ int swz(int r, int cc) {
  if constexpr (NP == 2) return cc ^ ((r >> 1) & 7);
  return (cc & ~3) | ((cc ^ (r >> 1)) & 3);
}

// Copy 16 bytes per lane from global address g into LDS at lds_addr + 16 * lane.
// lds_addr is the same in every lane.
__device__ __forceinline__ void lds_copy16(uint32_t lds_addr, const void* g) {
  const int m0 = __builtin_amdgcn_readfirstlane((int)lds_addr);
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" : : "s"(m0), "v"(g) : "memory", "m0");
}
// Wait until at most N vector memory operations of this wave are
// outstanding and all its LDS reads are done, then meet the workgroup.
template <int N>
__device__ __forceinline__ void wait_and_meet() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" : : "n"(N) : "memory");
}
constexpr int clamp63(int x) { return x < 63 ? x : 63; }
// N = BASE + e * NS for e in [0, E] (e is wave-uniform)
template <int BASE, int NS, int E>
__device__ __forceinline__ void wait_and_meet_sel(int e) {
  if constexpr (E == 0) {
    wait_and_meet<clamp63(BASE)>();
  } else {
    if (e == E)
      wait_and_meet<clamp63(BASE + E * NS)>();
    else
      wait_and_meet_sel<BASE, NS, E - 1>(e);
  }
}

// wait_and_meet<n> for a wave-uniform n in [LO, HI]
template <int LO, int HI>
__device__ __forceinline__ void wait_and_meet_rt(int n) {
  if constexpr (LO == HI) {
    wait_and_meet<LO>();
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (n <= MID)
      wait_and_meet_rt<LO, MID>(n);
    else
      wait_and_meet_rt<MID + 1, HI>(n);
  }
}

// A k-step record read from LDS, made wave-uniform.
struct Rec {
  int64_t a, b, c;
  int lda, ldb, rows, cols, kch, flags, kval, pad, ldc, c_buf, a_buf, b_buf;
};
__device__ __forceinline__ bf16x8 bf(u4 x) { return __builtin_bit_cast(bf16x8, x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ Rec read_rec(const unsigned char* p) {
  const u4 w0 = *reinterpret_cast<const u4*>(p);
  const u4 w1 = *reinterpret_cast<const u4*>(p + 16);
  const u4 w2 = *reinterpret_cast<const u4*>(p + 32);
  Rec r;
  r.a = (int64_t)((uint64_t)uni(w0.x) | ((uint64_t)uni(w0.y) << 32));
  r.b = (int64_t)((uint64_t)uni(w0.z) | ((uint64_t)uni(w0.w) << 32));
  r.lda = (int)uni(w1.x);
  r.ldb = (int)uni(w1.y);
  const uint32_t pk = uni(w1.z);
  r.rows = (int)(pk & 0xFF) + 1;
  r.cols = (int)((pk >> 8) & 0xFF) + 1;
  r.kch = (int)((pk >> 16) & 0xFF);
  r.flags = (int)(pk >> 24);
  const uint32_t pk2 = uni(w1.w);
  r.kval = (int)(pk2 & 0xFF);
  r.pad = (int)((pk2 >> 8) & 0xFF);
  r.c_buf = (int)(pk2 >> 16);
  r.c = (int64_t)((uint64_t)uni(w2.x) | ((uint64_t)uni(w2.y) << 32));
  r.ldc = (int)uni(w2.z);
  const uint32_t pk3 = uni(w2.w);
  r.a_buf = (int)(pk3 & 0xFFFF);
  r.b_buf = (int)(pk3 >> 16);
  return r;
}
}  // namespace

// Read by lanes whose k chunk lies past the operand rows, 16 bytes per lane
// (one shared address for a whole wave serialises in the cache); never written.
__device__ __attribute__((aligned(1024))) unsigned int g_stream_zero[64 * 4] = {};
// WGM x WGN waves, each owning a (BM / WGM) x (BN / WGN) part of the tile.
// Written by lanes outside the output tile (a 16-word slot per wave, so the
// lanes of one store stay within two cache lines; one word shared by the
// whole chip would serialise); never read.
constexpr int kSinkWgs = 4 * kStreamCUs;
__device__ __attribute__((aligned(256))) double g_stream_sink[kSinkWgs * 8 * 16];

template <int NP, typename TC, int BM, int BN, int S, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_planes_stream_kernel(const KStep* __restrict__ steps,
                                                                 const int64_t* __restrict__ wg_begin,
                                                                 void* const* __restrict__ ptrs,
                                                                 const int64_t* __restrict__ rowtab) {
  constexpr int NW = WGM * WGN, NT = 64 * NW;             // waves, lanes
  constexpr int WM = BM / WGM, WN = BN / WGN, SM = WM / 16, SN = WN / 16;
  constexpr int NC = 4 * NP;                            // 16-byte pieces per operand row
  constexpr int SLA = BM * NC, SLB = BN * NC;           // 16-byte slots of a stage
  constexpr int LPS = (SLA + SLB) / NT;                 // copies per lane per stage
  constexpr int RL = BM / NW / 2;                       // lanes per wave copying row offsets
  constexpr int BL = kStepBatch * 3 / NW;               // lanes per wave copying records
  constexpr int STB = (SLA + SLB) * 16;                 // stage bytes
  constexpr int REC = S * STB;                          // record ring
  constexpr int ROWS = REC + kStepRing * kStepBatch * 48;   // row-offset ring
  constexpr int LDSB = ROWS + S * BM * 8;
  constexpr int NS = SM * SN * 4;                       // stores per lane per tile
  static_assert(LDSB == stream_lds_bytes(NP, BM, BN, S), "LDS layout");
  static_assert(SLA % NT == 0 && SLB % NT == 0, "a copy round covers A or B slots only");
  static_assert(S >= 2 && S <= 16, "stages");
  static_assert(SM >= 1 && SN >= 1 && WM % 16 == 0 && WN % 16 == 0, "wave tiles of whole MFMA blocks");
  static_assert(RL >= 1 && RL * 2 * NW == BM && RL <= 64, "row-offset copy");
  static_assert(BL * NW == kStepBatch * 3, "record copy");
  __shared__ __attribute__((aligned(16))) unsigned char smem[LDSB];

  const int64_t first = wg_begin[blockIdx.x];
  const int n = (int)(wg_begin[blockIdx.x + 1] - first);
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(BST_LDS unsigned char*)smem;
  const unsigned char* gsteps = reinterpret_cast<const unsigned char*>(steps + first);
  // operand buffers of the current copies (re-read when a record names others)
  int a_buf = -1, b_buf = -1;
  const unsigned short* A = nullptr;
  const unsigned short* B = nullptr;
  const void* zero = g_stream_zero + 4 * lane;

  // record batch bi -> ring slot bi % kStepRing: 768 bytes, BL lanes per wave
  auto copy_batch = [&](int bi) {
    if (bi * kStepBatch < n && lane < BL)
      lds_copy16(lds0 + REC + (uint32_t)(bi % kStepRing) * (kStepBatch * 48) + wave * (BL * 16),
                 gsteps + (int64_t)bi * (kStepBatch * 48) + wave * (BL * 16) + lane * 16);
  };
  auto rec_ptr = [&](int v) -> const unsigned char* {
    return smem + REC + ((v / kStepBatch) % kStepRing) * (kStepBatch * 48) + (v % kStepBatch) * 48;
  };

  int tiles_in = 0, tiles_out = 0;   // tiles started by the copy cursor / written
  // copies of k-step v into stage v % S
  auto issue = [&](int v) {
    if (v % kStepBatch == 0) copy_batch(v / kStepBatch + 1);
    const Rec d = read_rec(rec_ptr(v));
    if ((d.flags & (kStepFirst | kStepRowmap)) == (kStepFirst | kStepRowmap)) {
      if (lane < RL)
        lds_copy16(lds0 + ROWS + (uint32_t)(tiles_in % S) * (BM * 8) + wave * (RL * 16),
                   rowtab + d.c + wave * (RL * 2) + lane * 2);
    }
    if (d.flags & kStepFirst) ++tiles_in;
    if (d.a_buf != a_buf) {
      a_buf = d.a_buf;
      A = static_cast<const unsigned short*>(ptrs[a_buf]);
    }
    if (d.b_buf != b_buf) {
      b_buf = d.b_buf;
      B = static_cast<const unsigned short*>(ptrs[b_buf]);
    }
    const uint32_t sb = lds0 + (uint32_t)(v % S) * STB;
#pragma unroll
    for (int i = 0; i < LPS; ++i) {
      const bool isA = i * NT < SLA;   // the same in every lane
      const int sl = isA ? i * NT + tid : i * NT - SLA + tid;   // slot within the operand
      const int r = sl / NC, cc = swz<NP>(r, sl % NC), kc = cc / NP;
      const int row = min(r, (isA ? d.rows : d.cols) - 1);
      // plane_at of (row, chunk kc, plane cc % NP): the row's pieces are contiguous
      const int64_t e = NP * (isA ? d.a + (int64_t)row * d.lda : d.b + (int64_t)row * d.ldb) + cc * 8;
      const void* g = kc < d.kch ? static_cast<const void*>((isA ? A : B) + e) : zero;
      lds_copy16(sb + (uint32_t)(i * NT * 16 + wave * 1024), g);
    }
  };

  flt4 acc[SM][SN];

  auto compute = [&](int u, const Rec& d) {
    const unsigned short* As = reinterpret_cast<const unsigned short*>(smem + (u % S) * STB);
    const unsigned short* Bs = As + BM * NC * 8;
    const int kc = lane >> 4;   // 8-element k chunk of this lane
    u4 a[NP][SM], b[NP][SN];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        const int r = wm * WM + i * 16 + (lane & 15);
        a[q][i] = *reinterpret_cast<const u4*>(As + r * NC * 8 + swz<NP>(r, kc * NP + q) * 8);
      }
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        const int r = wn * WN + j * 16 + (lane & 15);
        b[q][j] = *reinterpret_cast<const u4*>(Bs + r * NC * 8 + swz<NP>(r, kc * NP + q) * 8);
      }
    }
    // a partial last chunk (kval < 8 valid elements, in lanes of chunk
    // kch - 1): zero the elements past kval in both operands, so that
    // whatever the padding holds cannot reach the sums
    if (d.kval < 8) {
      const bool part = kc == d.kch - 1;
      auto mk = [&](int e) -> uint32_t {
        return !part ? ~0u : ((2 * e < d.kval ? 0xFFFFu : 0u) | (2 * e + 1 < d.kval ? 0xFFFF0000u : 0u));
      };
      const u4 m = {mk(0), mk(1), mk(2), mk(3)};
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int i = 0; i < SM; ++i) a[q][i] &= m;
#pragma unroll
        for (int j = 0; j < SN; ++j) b[q][j] &= m;
      }
    }
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        if constexpr (NP == 3) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[2][i]), bf(b[0][j]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[1][i]), bf(b[1][j]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[0][i]), bf(b[2][j]), acc[i][j], 0, 0, 0);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[1][i]), bf(b[0][j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[0][i]), bf(b[1][j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[0][i]), bf(b[0][j]), acc[i][j], 0, 0, 0);
      }
  };

  // every lane stores all SM * SN * 4 of its elements (exactly NS store
  // instructions per wave); lanes outside the tile store to the wave's
  // 16-word slot of the sink
  auto epilogue = [&](const Rec& d) {
    BST_G TC* C = (BST_G TC*)(ptrs[d.c_buf]);
    BST_G TC* sink = (BST_G TC*)(g_stream_sink + ((blockIdx.x % kSinkWgs) * 8 + wave) * 16 + (lane & 15));
    const int64_t* rmap = reinterpret_cast<const int64_t*>(smem + ROWS + (tiles_out % S) * (BM * 8));
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * WM + i * 16 + 4 * (lane >> 4) + r;
        int64_t rb;
        if (d.flags & kStepRowmap)
          rb = rmap[row];
        else
          rb = row < d.rows ? d.c + (int64_t)row * d.ldc : -1;
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const int col = wn * WN + j * 16 + (lane & 15);
          BST_G TC* p = (rb >= 0 && col < d.cols) ? C + rb + col : sink;
          *p = (TC)acc[i][j][r];
        }
      }
    ++tiles_out;
  };

  // prologue: first record batch, then the first S - 1 steps' copies
  copy_batch(0);
  wait_and_meet<0>();
  int v = 0;
  for (; v < n && v < S - 1; ++v) issue(v);
  unsigned epi = 0;   // bit k set: stores were issued k + 1 iterations ago (k < S - 1)
  constexpr unsigned kEpiMask = (1u << (S - 1)) - 1;
  int u = 0;
  // one tile per outer iteration (the accumulators start at zero), its
  // k-steps in the inner loop; copies run on across tile boundaries
  while (u < n) {
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) acc[i][j] = flt4{0, 0, 0, 0};
    Rec d;
    do {
      // outstanding after step u's copies: the copies of steps u+1 .. u+S-2
      // and the stores of the tiles finished since step u was issued
      if (n - 1 - u >= S - 2)
        wait_and_meet_sel<(S - 2) * LPS, NS, S - 1>(__builtin_popcount(epi));
      else
        wait_and_meet<0>();
      if (v < n) {
        issue(v);
        ++v;
      }
      d = read_rec(rec_ptr(u));
      compute(u, d);
      epi = (epi << 1) & kEpiMask;
      ++u;
    } while (!(d.flags & kStepLast) && u < n);
    epilogue(d);
    epi |= 1;
  }
}

// The same schedule on float64 operands held in the same padded layouts (one
// plane of doubles, positions = elements).  A k-step is 16 elements of a row:
// one 128-byte line, eight 16-byte pieces of two doubles, with the swizzle of
// the two-plane layout.  kch counts valid pieces (0..8) and kval the valid
// elements of piece kch - 1 (1 or 2).  v_mfma_f64_16x16x4f64 sums four k per
// instruction: lane group g = lane / 16 supplies element 4g + j of the step to
// MFMA j, so that every lane reads four consecutive elements of its row (two
// 16-byte LDS reads) for the step's four MFMAs.  The sum over the step is the
// same set of products in a fixed order, so results are bitwise repeatable.
template <int BM, int BN, int S, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_f64_stream_kernel(const KStep* __restrict__ steps,
                                                                     const int64_t* __restrict__ wg_begin,
                                                                     void* const* __restrict__ ptrs,
                                                                     const int64_t* __restrict__ rowtab) {
  constexpr int NW = WGM * WGN, NT = 64 * NW;
  constexpr int WM = BM / WGM, WN = BN / WGN, SM = WM / 16, SN = WN / 16;
  constexpr int NC = 8;                                 // 16-byte pieces per operand row and k-step
  constexpr int SLA = BM * NC, SLB = BN * NC;
  constexpr int LPS = (SLA + SLB) / NT;
  constexpr int RL = BM / NW / 2;
  constexpr int BL = kStepBatch * 3 / NW;
  constexpr int STB = (SLA + SLB) * 16;
  constexpr int REC = S * STB;
  constexpr int ROWS = REC + kStepRing * kStepBatch * 48;
  constexpr int LDSB = ROWS + S * BM * 8;
  constexpr int NS = SM * SN * 4;
  static_assert(LDSB == stream_lds_bytes(1, BM, BN, S), "LDS layout");
  static_assert(SLA % NT == 0 && SLB % NT == 0, "a copy round covers A or B slots only");
  static_assert(S >= 2 && S <= 16, "stages");
  static_assert(SM >= 1 && SN >= 1 && WM % 16 == 0 && WN % 16 == 0, "wave tiles of whole MFMA blocks");
  static_assert(RL >= 1 && RL * 2 * NW == BM && RL <= 64, "row-offset copy");
  static_assert(BL * NW == kStepBatch * 3, "record copy");
  __shared__ __attribute__((aligned(16))) unsigned char smem[LDSB];

  const int64_t first = wg_begin[blockIdx.x];
  const int n = (int)(wg_begin[blockIdx.x + 1] - first);
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(BST_LDS unsigned char*)smem;
  const unsigned char* gsteps = reinterpret_cast<const unsigned char*>(steps + first);
  int a_buf = -1, b_buf = -1;
  const double* A = nullptr;
  const double* B = nullptr;
  const void* zero = g_stream_zero + 4 * lane;

  auto copy_batch = [&](int bi) {
    if (bi * kStepBatch < n && lane < BL)
      lds_copy16(lds0 + REC + (uint32_t)(bi % kStepRing) * (kStepBatch * 48) + wave * (BL * 16),
                 gsteps + (int64_t)bi * (kStepBatch * 48) + wave * (BL * 16) + lane * 16);
  };
  auto rec_ptr = [&](int v) -> const unsigned char* {
    return smem + REC + ((v / kStepBatch) % kStepRing) * (kStepBatch * 48) + (v % kStepBatch) * 48;
  };

  int tiles_in = 0, tiles_out = 0;
  auto issue = [&](int v) {
    if (v % kStepBatch == 0) copy_batch(v / kStepBatch + 1);
    const Rec d = read_rec(rec_ptr(v));
    if ((d.flags & (kStepFirst | kStepRowmap)) == (kStepFirst | kStepRowmap)) {
      if (lane < RL)
        lds_copy16(lds0 + ROWS + (uint32_t)(tiles_in % S) * (BM * 8) + wave * (RL * 16),
                   rowtab + d.c + wave * (RL * 2) + lane * 2);
    }
    if (d.flags & kStepFirst) ++tiles_in;
    if (d.a_buf != a_buf) {
      a_buf = d.a_buf;
      A = static_cast<const double*>(ptrs[a_buf]);
    }
    if (d.b_buf != b_buf) {
      b_buf = d.b_buf;
      B = static_cast<const double*>(ptrs[b_buf]);
    }
    const uint32_t sb = lds0 + (uint32_t)(v % S) * STB;
#pragma unroll
    for (int i = 0; i < LPS; ++i) {
      const bool isA = i * NT < SLA;
      const int sl = isA ? i * NT + tid : i * NT - SLA + tid;
      const int r = sl / NC, cc = swz<2>(r, sl % NC);
      const int row = min(r, (isA ? d.rows : d.cols) - 1);
      const int64_t e = (isA ? d.a + (int64_t)row * d.lda : d.b + (int64_t)row * d.ldb) + cc * 2;
      const void* g = cc < d.kch ? static_cast<const void*>((isA ? A : B) + e) : zero;
      lds_copy16(sb + (uint32_t)(i * NT * 16 + wave * 1024), g);
    }
  };

  dbl4 acc[SM][SN];

  auto compute = [&](int u, const Rec& d) {
    const unsigned char* As = smem + (u % S) * STB;
    const unsigned char* Bs = As + BM * NC * 16;
    const int g = lane >> 4;   // this lane's elements 4g .. 4g + 3 of the step
    dbl2 a[SM][2], b[SN][2];
#pragma unroll
    for (int i = 0; i < SM; ++i) {
      const int r = wm * WM + i * 16 + (lane & 15);
#pragma unroll
      for (int h = 0; h < 2; ++h) a[i][h] = *reinterpret_cast<const dbl2*>(As + (r * NC + swz<2>(r, 2 * g + h)) * 16);
    }
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int r = wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int h = 0; h < 2; ++h) b[j][h] = *reinterpret_cast<const dbl2*>(Bs + (r * NC + swz<2>(r, 2 * g + h)) * 16);
    }
    // a partial last piece (one valid element): zero its second element in
    // both operands, so that whatever the padding holds cannot reach the sums
    if (d.kval < 2) {
      const int p = d.kch - 1;   // piece index; this lane holds pieces 2g, 2g + 1
      if ((p >> 1) == g) {
        const int h = p & 1;
#pragma unroll
        for (int i = 0; i < SM; ++i) a[i][h].y = 0.0;
#pragma unroll
        for (int j = 0; j < SN; ++j) b[j][h].y = 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const double av = (q & 1) ? a[i][q >> 1].y : a[i][q >> 1].x;
          const double bv = (q & 1) ? b[j][q >> 1].y : b[j][q >> 1].x;
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[i][j], 0, 0, 0);
        }
  };

  // float64 accumulators: register r of lane l holds row 4r + l / 16,
  // column l % 16 of the 16 x 16 block
  auto epilogue = [&](const Rec& d) {
    BST_G double* C = (BST_G double*)(ptrs[d.c_buf]);
    BST_G double* sink = (BST_G double*)(g_stream_sink + ((blockIdx.x % kSinkWgs) * 8 + wave) * 16 + (lane & 15));
    const int64_t* rmap = reinterpret_cast<const int64_t*>(smem + ROWS + (tiles_out % S) * (BM * 8));
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * WM + i * 16 + 4 * r + (lane >> 4);
        int64_t rb;
        if (d.flags & kStepRowmap)
          rb = rmap[row];
        else
          rb = row < d.rows ? d.c + (int64_t)row * d.ldc : -1;
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          const int col = wn * WN + j * 16 + (lane & 15);
          BST_G double* p = (rb >= 0 && col < d.cols) ? C + rb + col : sink;
          *p = acc[i][j][r];
        }
      }
    ++tiles_out;
  };

  copy_batch(0);
  wait_and_meet<0>();
  int v = 0;
  for (; v < n && v < S - 1; ++v) issue(v);
  unsigned epi = 0;
  constexpr unsigned kEpiMask = (1u << (S - 1)) - 1;
  int u = 0;
  while (u < n) {
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) acc[i][j] = dbl4{0, 0, 0, 0};
    Rec d;
    do {
      if (n - 1 - u >= S - 2)
        wait_and_meet_sel<(S - 2) * LPS, NS, S - 1>(__builtin_popcount(epi));
      else
        wait_and_meet<0>();
      if (v < n) {
        issue(v);
        ++v;
      }
      d = read_rec(rec_ptr(u));
      compute(u, d);
      epi = (epi << 1) & kEpiMask;
      ++u;
    } while (!(d.flags & kStepLast) && u < n);
    epilogue(d);
    epi |= 1;
  }
}

// Float64 shapes (gemm_planes_shapes(1), all of kind 3): bm, bn, stages,
// waves along M, waves along N.
#define BST_STREAM64_SHAPES(X) \
  X(64, 64, 3, 2, 2)           \
  X(128, 64, 3, 2, 2)          \
  X(64, 128, 3, 2, 2)          \
  X(128, 128, 3, 2, 4)         \
  X(256, 128, 3, 4, 2)         \
  X(128, 256, 3, 2, 4)         \
  X(64, 64, 2, 2, 2)           \
  X(128, 64, 2, 2, 2)          \
  X(64, 128, 2, 2, 2)          \
  X(128, 128, 2, 2, 4)

// Shapes of kind 3 in gemm_planes_shapes(np), instantiated here
// (np, bm, bn, stages, waves along M, waves along N).
#define BST_STREAM_SHAPES(X) \
  X(2, 128, 64, 3, 2, 2)     \
  X(2, 64, 128, 3, 2, 2)     \
  X(2, 128, 128, 3, 2, 4)    \
  X(2, 128, 256, 3, 2, 4)    \
  X(2, 256, 128, 3, 4, 2)    \
  X(2, 256, 64, 3, 4, 2)     \
  X(2, 64, 192, 3, 1, 4)     \
  X(2, 64, 192, 2, 1, 4)     \
  X(2, 128, 192, 3, 2, 4)    \
  X(2, 128, 128, 2, 2, 4)    \
  X(2, 128, 64, 2, 2, 2)     \
  X(2, 64, 128, 2, 2, 2)     \
  X(2, 32, 192, 2, 1, 4)     \
  X(3, 64, 64, 3, 2, 2)      \
  X(3, 128, 128, 3, 2, 4)

hipError_t launch_gemm_planes_stream(const StreamLaunch& g, hipStream_t s) {
  if (g.nwg <= 0) return hipSuccess;
  if (g.nwg > 0x7FFFFFFF) return hipErrorInvalidValue;
  const TileShape& sh = gemm_planes_shapes(g.np)[g.tile];
  if (sh.direct != 3) return hipErrorInvalidValue;
  const dim3 grid((unsigned)g.nwg);
  if (g.np == 1) {
    if (g.tc != ElemType::F64) return hipErrorInvalidValue;
#define BST_LAUNCH64(BM_, BN_, S_, WGM_, WGN_)                                                              \
  if (sh.bm == BM_ && sh.bn == BN_ && sh.stages == S_ && sh.waves == WGM_ * WGN_) {                        \
    hipLaunchKernelGGL((gemm_f64_stream_kernel<BM_, BN_, S_, WGM_, WGN_>), grid, dim3(64 * WGM_ * WGN_), 0, s, \
                       g.steps, g.wg_begin, g.ptrs, g.rowtab);                                            \
    return hipGetLastError();                                                                             \
  }
    BST_STREAM64_SHAPES(BST_LAUNCH64)
#undef BST_LAUNCH64
    return hipErrorInvalidValue;
  }
#define BST_LAUNCH(NP_, BM_, BN_, S_, WGM_, WGN_)                                                          \
  if (g.np == NP_ && sh.bm == BM_ && sh.bn == BN_ && sh.stages == S_ && sh.waves == WGM_ * WGN_) {        \
    const dim3 block(64 * WGM_ * WGN_);                                                                    \
    if (g.tc == ElemType::F32)                                                                            \
      hipLaunchKernelGGL((gemm_planes_stream_kernel<NP_, float, BM_, BN_, S_, WGM_, WGN_>), grid, block, 0, \
                         s, g.steps, g.wg_begin, g.ptrs, g.rowtab);                            \
    else                                                                                                  \
      hipLaunchKernelGGL((gemm_planes_stream_kernel<NP_, double, BM_, BN_, S_, WGM_, WGN_>), grid, block, \
                         0, s, g.steps, g.wg_begin, g.ptrs, g.rowtab);                         \
    return hipGetLastError();                                                                             \
  }
  BST_STREAM_SHAPES(BST_LAUNCH)
#undef BST_LAUNCH
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------
// L.psi fused with the two-site MPO apply (two bfloat16 planes, BF16x3).
//
// One tile is 64 rows (a index) x 64 columns (b' index) of one MPO task
// (a sector, b' sector).  For every input channel p = (w1, t1, t2) of the
// task, T1_p = L_(a,w1) . psi_(a',t1,t2,b') over the contracted sector a'
// (a' = a - w1) is accumulated in registers exactly as the L.psi GEMM
// forms it (same k-steps, same products and order), then folded into the
// task's outputs: out_o += h[o][p] T1_p over the nonzero coefficients in
// increasing p, as the MPO apply adds them.  At the tile's end every output
// is split into two bfloat16 planes and written to T3, so T1 never goes
// through memory.  The records are those of the pipelined kernel; per
// record pad = p, flags add kStepPlaneEnd on the last step of a channel,
// c_buf = the task's output count, c = coefficient offset (low 32 bits) and
// output-plane offset (high 32 bits), ldc = first row | first column << 16.
// At a tile's first step the class's dense coefficients (NMAX x NMAX
// floats) and its output planes (NMAX HPlane records) are copied into an LDS
// ring slot beside the operand stages.
// ------------------------------------------------------------------------
template <int NMAX>
__global__ __launch_bounds__(512) void lh_fused_kernel(const KStep* __restrict__ steps,
                                                       const int64_t* __restrict__ wg_begin,
                                                       void* const* __restrict__ ptrs,
                                                       const float* __restrict__ coef,
                                                       const HPlane* __restrict__ planes, int out_slot) {
  constexpr int NP = 2, BM = 64, BN = 64, S = 3, WGM = 2, WGN = 4;
  constexpr int NW = WGM * WGN, NT = 64 * NW;
  constexpr int WM = BM / WGM, WN = BN / WGN, SM = WM / 16, SN = WN / 16;
  constexpr int NC = 4 * NP;
  constexpr int SLA = BM * NC, SLB = BN * NC;
  constexpr int LPS = (SLA + SLB) / NT;
  constexpr int BL = kStepBatch * 3 / NW;
  constexpr int STB = (SLA + SLB) * 16;
  constexpr int REC = S * STB;
  constexpr int TABS = REC + kStepRing * kStepBatch * 48;
  constexpr int TAB = NMAX * NMAX * 4 + NMAX * 16;
  constexpr int LDSB = TABS + S * TAB;
  static_assert(SLA % NT == 0 && SLB % NT == 0, "a copy round covers A or B slots only");
  static_assert(BL * NW == kStepBatch * 3, "record copy");
  static_assert(NMAX * NMAX / 4 <= 64 && NMAX <= 64, "table copies: one wave each");
  static_assert(LDSB == lh_fused_lds_bytes(NMAX), "LDS layout");
  __shared__ __attribute__((aligned(16))) unsigned char smem[LDSB];

  const int64_t first = wg_begin[blockIdx.x];
  const int n = (int)(wg_begin[blockIdx.x + 1] - first);
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(BST_LDS unsigned char*)smem;
  const unsigned char* gsteps = reinterpret_cast<const unsigned char*>(steps + first);
  int a_buf = -1, b_buf = -1;
  const unsigned short* A = nullptr;
  const unsigned short* B = nullptr;
  const void* zero = g_stream_zero + 4 * lane;
  BST_G unsigned short* T3 = (BST_G unsigned short*)(ptrs[out_slot]);
  BST_G unsigned short* sink =
      (BST_G unsigned short*)(g_stream_sink + ((blockIdx.x % kSinkWgs) * 8 + wave) * 16) + (lane & 15);

  auto copy_batch = [&](int bi) {
    if (bi * kStepBatch < n && lane < BL)
      lds_copy16(lds0 + REC + (uint32_t)(bi % kStepRing) * (kStepBatch * 48) + wave * (BL * 16),
                 gsteps + (int64_t)bi * (kStepBatch * 48) + wave * (BL * 16) + lane * 16);
  };
  auto rec_ptr = [&](int v) -> const unsigned char* {
    return smem + REC + ((v / kStepBatch) % kStepRing) * (kStepBatch * 48) + (v % kStepBatch) * 48;
  };

  int tiles_in = 0, tiles_out = 0;
  auto issue = [&](int v) {
    if (v % kStepBatch == 0) copy_batch(v / kStepBatch + 1);
    const Rec d = read_rec(rec_ptr(v));
    if (d.flags & kStepFirst) {
      // the tile's coefficient block and output planes into its ring slot
      const uint32_t tb = lds0 + TABS + (uint32_t)(tiles_in % S) * TAB;
      const int64_t coff = (int64_t)(uint32_t)(d.c & 0xFFFFFFFF), poff = d.c >> 32;
      if (wave == 0 && lane < NMAX * NMAX / 4) lds_copy16(tb, coef + coff + 4 * lane);
      if (wave == 1 && lane < NMAX) lds_copy16(tb + NMAX * NMAX * 4, planes + poff + lane);
      ++tiles_in;
    }
    if (d.a_buf != a_buf) {
      a_buf = d.a_buf;
      A = static_cast<const unsigned short*>(ptrs[a_buf]);
    }
    if (d.b_buf != b_buf) {
      b_buf = d.b_buf;
      B = static_cast<const unsigned short*>(ptrs[b_buf]);
    }
    const uint32_t sb = lds0 + (uint32_t)(v % S) * STB;
#pragma unroll
    for (int i = 0; i < LPS; ++i) {
      const bool isA = i * NT < SLA;
      const int sl = isA ? i * NT + tid : i * NT - SLA + tid;
      const int r = sl / NC, cc = swz<NP>(r, sl % NC), kc = cc / NP;
      const int row = min(r, (isA ? d.rows : d.cols) - 1);
      const int64_t e = NP * (isA ? d.a + (int64_t)row * d.lda : d.b + (int64_t)row * d.ldb) + cc * 8;
      const void* g = kc < d.kch ? static_cast<const void*>((isA ? A : B) + e) : zero;
      lds_copy16(sb + (uint32_t)(i * NT * 16 + wave * 1024), g);
    }
  };

  flt4 acc[SM][SN];
  flt4 out[NMAX][SM][SN];

  auto compute = [&](int u, const Rec& d) {
    const unsigned short* As = reinterpret_cast<const unsigned short*>(smem + (u % S) * STB);
    const unsigned short* Bs = As + BM * NC * 8;
    const int kc = lane >> 4;
    u4 a[NP][SM], b[NP][SN];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        const int r = wm * WM + i * 16 + (lane & 15);
        a[q][i] = *reinterpret_cast<const u4*>(As + r * NC * 8 + swz<NP>(r, kc * NP + q) * 8);
      }
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        const int r = wn * WN + j * 16 + (lane & 15);
        b[q][j] = *reinterpret_cast<const u4*>(Bs + r * NC * 8 + swz<NP>(r, kc * NP + q) * 8);
      }
    }
    if (d.kval < 8) {
      const bool part = kc == d.kch - 1;
      auto mk = [&](int e) -> uint32_t {
        return !part ? ~0u : ((2 * e < d.kval ? 0xFFFFu : 0u) | (2 * e + 1 < d.kval ? 0xFFFF0000u : 0u));
      };
      const u4 m = {mk(0), mk(1), mk(2), mk(3)};
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int i = 0; i < SM; ++i) a[q][i] &= m;
#pragma unroll
        for (int j = 0; j < SN; ++j) b[q][j] &= m;
      }
    }
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[1][i]), bf(b[0][j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[0][i]), bf(b[1][j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(a[0][i]), bf(b[0][j]), acc[i][j], 0, 0, 0);
      }
  };

  // T1_p (acc) into the outputs: out_o += h[o][p] T1_p for nonzero h
  auto fold = [&](const Rec& d) {
    const float* ct = reinterpret_cast<const float*>(smem + TABS + (tiles_out % S) * TAB);
    const int p = d.pad, nout = d.c_buf;
#pragma unroll
    for (int o = 0; o < NMAX; ++o) {
      const float hv = o < nout ? ct[o * NMAX + p] : 0.0f;
      if (hv != 0.0f) {
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
          for (int j = 0; j < SN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[o][i][j][r] += hv * acc[i][j][r];
      }
    }
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) acc[i][j] = flt4{0, 0, 0, 0};
  };

  // every output o < nout: 2 * SM * SN * 4 stores per lane (lanes outside
  // the tile to the sink); returns the store count
  auto epilogue = [&](const Rec& d) -> int {
    const HPlane* qp = reinterpret_cast<const HPlane*>(smem + TABS + (tiles_out % S) * TAB + NMAX * NMAX * 4);
    const int nout = d.c_buf, m0 = d.ldc & 0xFFFF, n0 = (int)((uint32_t)d.ldc >> 16);
#pragma unroll
    for (int o = 0; o < NMAX; ++o) {
      if (o < nout) {
        const HPlane q = qp[o];
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = wm * WM + i * 16 + 4 * (lane >> 4) + r;
#pragma unroll
            for (int j = 0; j < SN; ++j) {
              const int col = wn * WN + j * 16 + (lane & 15);
              const bool in = row < d.rows && col < d.cols;
              const int64_t at = q.off + (int64_t)(m0 + row) * q.rowstride + (n0 + col);
              const float yf = out[o][i][j][r];
              unsigned int u = __float_as_uint(yf);
              const unsigned short h0 = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
              const float r1 = yf - __uint_as_float((unsigned int)h0 << 16);
              u = __float_as_uint(r1);
              const unsigned short h1 = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
              *(in ? T3 + plane_at(NP, at, 0) : sink) = h0;
              *(in ? T3 + plane_at(NP, at, 1) : sink) = h1;
            }
          }
      }
    }
#pragma unroll
    for (int o = 0; o < NMAX; ++o)
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) out[o][i][j] = flt4{0, 0, 0, 0};
    ++tiles_out;
    return nout * 2 * SM * SN * 4;
  };

#pragma unroll
  for (int o = 0; o < NMAX; ++o)
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) out[o][i][j] = flt4{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = flt4{0, 0, 0, 0};

  copy_batch(0);
  wait_and_meet<0>();
  int v = 0;
  for (; v < n && v < S - 1; ++v) issue(v);
  // store instructions issued in the last S - 1 iterations (newest first)
  int st0 = 0, st1 = 0;
  for (int u = 0; u < n; ++u) {
    // outstanding after step u's copies: the copies of steps u+1 .. u+S-2
    // and the stores issued since step u was issued (a lower bound of the
    // memory operations issued after step u's copies)
    if (n - 1 - u >= S - 2) {
      const int w = (S - 2) * LPS + st0 + st1;
      wait_and_meet_rt<0, 63>(w < 63 ? w : 63);
    } else {
      wait_and_meet<0>();
    }
    if (v < n) {
      issue(v);
      ++v;
    }
    const Rec d = read_rec(rec_ptr(u));
    compute(u, d);
    if (d.flags & kStepPlaneEnd) fold(d);
    st1 = st0;
    st0 = (d.flags & kStepLast) ? epilogue(d) : 0;
  }
}

hipError_t launch_lh_fused(const LhFusedLaunch& f, hipStream_t s) {
  if (f.nwg <= 0) return hipSuccess;
  if (f.nwg > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)f.nwg), block(512);
  if (f.nmax == 8)
    hipLaunchKernelGGL(lh_fused_kernel<8>, grid, block, 0, s, f.steps, f.wg_begin, f.ptrs, f.coef, f.planes,
                       f.out_slot);
  else if (f.nmax == 16)
    hipLaunchKernelGGL(lh_fused_kernel<16>, grid, block, 0, s, f.steps, f.wg_begin, f.ptrs, f.coef, f.planes,
                       f.out_slot);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace bst

// Bandwidth-bound kernels: block permute, the two-site MPO (h = W1.W2)
// apply, and the float64 vector kernels of Lanczos.  All are HBM-bound; they
// read and write each element once, coalesced along the fastest index, with
// LDS used to turn transposes into coalesced reads and writes.
#include "bst_internal.h"

namespace bst {

// ------------------------------------------------------------------------
// Block permute (Sec. "Permute", App. "Contiguous")
// ------------------------------------------------------------------------
static_assert(kPermRows <= 256 * 17, "row offsets share the transpose tile's LDS");

// Streaming 16-byte access when the address is 16-byte aligned, else two
// 8-byte accesses (block offsets and strides may be odd).
typedef double dbl2v __attribute__((ext_vector_type(2)));

// One transposing tile of TY x TX elements (TY = 4096 / TX) over (pdim,
// last): read as pairs of consecutive input columns, written as pairs of
// consecutive output positions (input rows) through LDS rows padded by one
// element.  Odd addresses fall back to 8-byte accesses.
template <int TX>
__device__ __forceinline__ void permute_tile(const PermJob& j, const PermWork& w, const BST_G double* __restrict__ in,
                                             BST_G double* __restrict__ out, double* lds) {
  constexpr int TY = 4096 / TX, LD = TX + 1;
  const int r = j.rank, tid = threadIdx.x;
  const int p = j.pdim;
  int64_t rem = w.batch, ib = 0, ob = 0;
  for (int d = r - 1; d >= 0; --d) {
    if (d == p || d == r - 1) continue;
    const int64_t ext = j.shape[d];
    const int64_t idx = rem % ext;
    rem /= ext;
    ib += idx * j.istride[d];
    ob += idx * j.ostride[d];
  }
  const int np = j.shape[p], nl = j.shape[r - 1];
  const int64_t isp = j.istride[p], osl = j.ostride[r - 1];
#pragma unroll
  for (int k = 0; k < 2048 / 256; ++k) {
    const int e = tid + 256 * k;
    const int y = e / (TX / 2), x = 2 * (e % (TX / 2));
    const int gy = w.t0 + y, gx = w.t1 + x;
    if (gy < np && gx < nl) {
      const BST_G double* src = in + ib + gy * isp + gx;
      if (gx + 1 < nl && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const dbl2v v = __builtin_nontemporal_load(reinterpret_cast<const BST_G dbl2v*>(src));
        lds[y * LD + x] = v.x;
        lds[y * LD + x + 1] = v.y;
      } else {
        lds[y * LD + x] = src[0];
        if (gx + 1 < nl) lds[y * LD + x + 1] = src[1];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2048 / 256; ++k) {
    const int e = tid + 256 * k;
    const int x = e / (TY / 2), y = 2 * (e % (TY / 2));
    const int gy = w.t0 + y, gx = w.t1 + x;
    if (gy < np && gx < nl) {
      BST_G double* dst = out + ob + gy + gx * osl;
      if (gy + 1 < np && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        dbl2v v;
        v.x = lds[y * LD + x];
        v.y = lds[(y + 1) * LD + x];
        __builtin_nontemporal_store(v, reinterpret_cast<BST_G dbl2v*>(dst));
      } else {
        dst[0] = lds[y * LD + x];
        if (gy + 1 < np) dst[1] = lds[(y + 1) * LD + x];
      }
    }
  }
}

__global__ __launch_bounds__(256) void permute_kernel(const PermJob* __restrict__ jobs,
                                                      const PermWork* __restrict__ work,
                                                      void* const* __restrict__ ptrs) {
  __shared__ double tile[1][256 * 17];   // the largest tile: 256 x (16 + 1)
  const PermWork w = work[blockIdx.x];
  const PermJob& j = jobs[w.job];
  const BST_G double* __restrict__ in = (const BST_G double*)(ptrs[j.in_buf]) + j.in_off;
  BST_G double* __restrict__ out = (BST_G double*)(ptrs[j.out_buf]) + j.out_off;
  const int r = j.rank;
  const int tid = threadIdx.x;
  if (w.kind == 0) {
    // fastest dim kept: rows w.batch .. w.batch + w.t0 - 1 are copied whole.
    // The rows' output offsets go to LDS first; then the block's element
    // pairs are spread over all lanes regardless of the row length.
    int64_t* orow = reinterpret_cast<int64_t*>(&tile[0][0]);   // kPermRows <= tile size
    const int64_t last = j.shape[r - 1];
    const int nrow = w.t0;
    for (int q = tid; q < nrow; q += 256) {
      int64_t rem = w.batch + q, ob = 0;
      for (int d = r - 2; d >= 0; --d) {
        const int64_t ext = j.shape[d];
        const int64_t idx = rem % ext;
        rem /= ext;
        ob += idx * j.ostride[d];
      }
      orow[q] = ob;
    }
    __syncthreads();
    const int64_t npair = (last + 1) / 2;
    for (int64_t e = tid; e < (int64_t)nrow * npair; e += 256) {
      const int64_t q = e / npair, c = 2 * (e - q * npair);
      const BST_G double* src = in + (w.batch + q) * last + c;
      BST_G double* dst = out + orow[q] + c;
      if (c + 1 < last && ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
        __builtin_nontemporal_store(__builtin_nontemporal_load(reinterpret_cast<const BST_G dbl2v*>(src)),
                                    reinterpret_cast<BST_G dbl2v*>(dst));
      } else {
        dst[0] = src[0];
        if (c + 1 < last) dst[1] = src[1];
      }
    }
    return;
  }
  // transposing job: a tile over (pdim, last) at origin (t0, t1), 64 x 64,
  // or 128 x 32 / 256 x 16 for a narrow last strip of the last dim
  if (w.kind == 1) permute_tile<64>(j, w, in, out, tile[0]);
  else if (w.kind == 2) permute_tile<32>(j, w, in, out, tile[0]);
  else permute_tile<16>(j, w, in, out, tile[0]);
}

// Complex B operand of a complex contraction, expanded for a real GEMM:
// element (k, n) = br + i bi becomes the 2 x 2 real block
// out[k][c][n][c'] = [[br, bi], [-bi, br]][c][c'].
__global__ __launch_bounds__(256) void expand_kernel(const ExpandJob* __restrict__ jobs,
                                                     const ExpandWork* __restrict__ work,
                                                     void* const* __restrict__ ptrs) {
  const ExpandWork w = work[blockIdx.x];
  const ExpandJob j = jobs[w.job];
  const double* __restrict__ in = static_cast<const double*>(ptrs[j.in_buf]) + j.in_off;
  double* __restrict__ out = static_cast<double*>(ptrs[j.out_buf]) + j.out_off;
  const int64_t total = (int64_t)j.K * j.N;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int64_t idx = (int64_t)w.start + e;
    if (idx >= total) break;
    const int64_t k = idx / j.N, n = idx % j.N;
    const double br = in[2 * idx], bi = in[2 * idx + 1];
    double* o0 = out + ((k * 2) * j.N + n) * 2;
    double* o1 = out + ((k * 2 + 1) * j.N + n) * 2;
    o0[0] = br;
    o0[1] = bi;
    o1[0] = -bi;
    o1[1] = br;
  }
}

hipError_t launch_expand(const ExpandLaunch& l, hipStream_t s) {
  if (l.nwork <= 0) return hipSuccess;
  if (l.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(expand_kernel, dim3((unsigned)l.nwork), dim3(256), 0, s, l.jobs, l.work, l.ptrs);
  return hipGetLastError();
}

hipError_t launch_permute(const PermLaunch& p, hipStream_t s) {
  if (p.nwork <= 0) return hipSuccess;
  if (p.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)p.nwork), dim3(256), 0, s, p.jobs, p.work,
                     p.ptrs);
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// Two-site MPO apply.  For every pair (a-sector, b'-sector) the T1 planes
// (w1 channel, t1, t2) map to the T3 planes (s1, s2, w3) through the small
// matrix h[o][i] = sum_w2 W1[w1,s1,t1,w2] W2[w2,s2,t2,w3] (Sec. "Benchmarks",
// Fig. Hpsi_fig: the two W's form the two-site operator h).
// ------------------------------------------------------------------------
// Every entry of a coefficient row (class, output o) is the sum of its W1*W2
// terms in a fixed order; the row is written dense (coef64/coef32) and
// compacted to its nonzero entries in increasing input order (cnt, idx,
// val64, val32) for the sparse apply.
__global__ __launch_bounds__(256) void hcoef_kernel(const HTerm* __restrict__ terms,
                                                    const int32_t* __restrict__ entry_begin,
                                                    int64_t nentries, int nmax,
                                                    void* const* __restrict__ ptrs,
                                                    double* __restrict__ c64,
                                                    float* __restrict__ c32,
                                                    int32_t* __restrict__ cnt,
                                                    int32_t* __restrict__ idx,
                                                    double* __restrict__ v64,
                                                    float* __restrict__ v32) {
  // one lane per entry, then one lane per row compacts the row (nmax
  // divides 256, so a workgroup holds whole rows)
  __shared__ double cs[256];
  const int tid = threadIdx.x;
  const int64_t e = (int64_t)blockIdx.x * 256 + tid;
  double sum = 0.0;
  if (e < nentries) {
    for (int32_t k = entry_begin[e]; k < entry_begin[e + 1]; ++k) {
      const HTerm t = terms[k];
      const double w1 = ((const BST_G double*)(ptrs[t.w1_buf]))[t.w1_off];
      const double w2 = ((const BST_G double*)(ptrs[t.w2_buf]))[t.w2_off];
      sum += w1 * w2;
    }
    c64[e] = sum;
    c32[e] = (float)sum;
  }
  cs[tid] = sum;
  __syncthreads();
  const int rpb = 256 / nmax;
  if (tid >= rpb) return;
  const int64_t row = (int64_t)blockIdx.x * rpb + tid;
  if (row * nmax >= nentries) return;
  int32_t n = 0;
  for (int i = 0; i < nmax; ++i) {
    const double v = cs[tid * nmax + i];
    if (v != 0.0) {
      idx[row * nmax + n] = i;
      v64[row * nmax + n] = v;
      v32[row * nmax + n] = (float)v;
      ++n;
    }
  }
  cnt[row] = n;
}

hipError_t launch_hcoef(const HCoefLaunch& c, hipStream_t s) {
  if (c.nentries <= 0) return hipSuccess;
  if (c.nmax <= 0 || 256 % c.nmax != 0 || c.nentries % c.nmax != 0) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((c.nentries + 255) / 256);
  hipLaunchKernelGGL(hcoef_kernel, dim3(blocks), dim3(256), 0, s, c.terms, c.entry_begin, c.nentries,
                     c.nmax, c.ptrs, c.coef64, c.coef32, c.cnt, c.idx, c.val64, c.val32);
  return hipGetLastError();
}

// Sparse two-site MPO apply: each lane stages its site's nin inputs in LDS
// (one column per lane, no bank conflicts) and runs only the nonzero terms
// of its class.  The terms of an output are added in increasing input order,
// so the result equals the dense product bit for bit.
template <typename T, int NMAX, int NP, bool O32>
__global__ __launch_bounds__(256) void happly_sparse_kernel(const HTask* __restrict__ tasks,
                                                            const HPlane* __restrict__ planes,
                                                            const HWork* __restrict__ work,
                                                            void* const* __restrict__ ptrs,
                                                            const int32_t* __restrict__ cnt,
                                                            const int32_t* __restrict__ idx,
                                                            const T* __restrict__ val) {
  __shared__ T xs[NMAX][256];
  __shared__ T sv[NMAX * NMAX];
  __shared__ int32_t si[NMAX * NMAX];
  __shared__ int32_t sc[NMAX];
  __shared__ HPlane pl[2 * NMAX];
  const HWork w = work[blockIdx.x];
  const HTask t = tasks[w.task];
  const int tid = threadIdx.x;
  const int64_t cbase = (int64_t)t.cls * NMAX;
  for (int e = tid; e < NMAX * NMAX; e += 256) {
    sv[e] = val[cbase * NMAX + e];
    si[e] = idx[cbase * NMAX + e];
  }
  for (int e = tid; e < NMAX; e += 256) sc[e] = cnt[cbase + e];
  for (int e = tid; e < t.nin + t.nout; e += 256) pl[e] = planes[t.plane_begin + e];
  __syncthreads();
  const int site = w.site0 + tid;
  if (site >= t.rows * t.cols) return;
  const int i = site / t.cols, jc = site % t.cols;
  const BST_G T* __restrict__ in = (const BST_G T*)(ptrs[t.in_buf]);
  // all input loads in flight at once, then staged (each lane reads back
  // only its own column, so no barrier is needed)
  T xr[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if constexpr (O32)
      xr[k] = (k < t.nin) ? in[(uint32_t)pl[k].off + (uint32_t)i * (uint32_t)pl[k].rowstride + (uint32_t)jc]
                          : T(0);
    else
      xr[k] = (k < t.nin) ? in[pl[k].off + (int64_t)i * pl[k].rowstride + jc] : T(0);
  }
#pragma unroll
  for (int k = 0; k < NMAX; ++k) xs[k][tid] = xr[k];
  for (int o = 0; o < t.nout; ++o) {
    T y = 0;
    const int n = sc[o];
    for (int e = 0; e < n; ++e) y += sv[o * NMAX + e] * xs[si[o * NMAX + e]][tid];
    const HPlane q = pl[t.nin + o];
    using IX = typename std::conditional<O32, uint32_t, int64_t>::type;
    const IX at = O32 ? (IX)((uint32_t)q.off + (uint32_t)i * (uint32_t)q.rowstride + (uint32_t)jc)
                      : (IX)(q.off + (int64_t)i * q.rowstride + jc);
    if constexpr (NP == 0) {
      ((BST_G T*)(ptrs[t.out_buf]))[at] = y;
    } else {
      BST_G unsigned short* out = (BST_G unsigned short*)(ptrs[t.out_buf]);
      const float yf = (float)y;
      unsigned int u = __float_as_uint(yf);
      const unsigned short h0 = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
      const float r1 = yf - __uint_as_float((unsigned int)h0 << 16);
      u = __float_as_uint(r1);
      const unsigned short h1 = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
      out[plane_at(NP, at, 0)] = h0;
      out[plane_at(NP, at, 1)] = h1;
      if constexpr (NP == 3) {
        const float r2 = r1 - __uint_as_float((unsigned int)h1 << 16);
        u = __float_as_uint(r2);
        out[plane_at(NP, at, 2)] = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
      }
    }
  }
}

hipError_t launch_happly_sparse(const HApplyLaunch& h, hipStream_t s) {
  if (h.nwork <= 0) return hipSuccess;
  if (h.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  dim3 grid((unsigned)h.nwork), block(256);
#define BST_HS(T_, N_, P_)                                                                     \
  if (h.nmax == N_ && h.np == P_) {                                                            \
    if (h.off32)                                                                               \
      hipLaunchKernelGGL((happly_sparse_kernel<T_, N_, P_, true>), grid, block, 0, s, h.tasks,   \
                         h.planes, h.work, h.ptrs, h.cnt, h.idx, reinterpret_cast<const T_*>(h.val)); \
    else                                                                                       \
      hipLaunchKernelGGL((happly_sparse_kernel<T_, N_, P_, false>), grid, block, 0, s, h.tasks,  \
                         h.planes, h.work, h.ptrs, h.cnt, h.idx, reinterpret_cast<const T_*>(h.val)); \
    return hipGetLastError();                                                                  \
  }
  if (h.t == ElemType::F64) {
    BST_HS(double, 8, 0) BST_HS(double, 16, 0)
  } else {
    BST_HS(float, 8, 0) BST_HS(float, 16, 0) BST_HS(float, 8, 2) BST_HS(float, 16, 2)
    BST_HS(float, 8, 3) BST_HS(float, 16, 3)
  }
#undef BST_HS
  return hipErrorInvalidValue;
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) void happly_kernel(const HTask* __restrict__ tasks,
                                                     const HPlane* __restrict__ planes,
                                                     const HWork* __restrict__ work,
                                                     void* const* __restrict__ ptrs,
                                                     const T* __restrict__ coef) {
  __shared__ T cf[NMAX * NMAX];
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
  const BST_G T* __restrict__ in = (const BST_G T*)(ptrs[t.in_buf]);
  BST_G T* __restrict__ out = (BST_G T*)(ptrs[t.out_buf]);
  T x[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k)
    x[k] = (k < t.nin) ? in[pl[k].off + (int64_t)i * pl[k].rowstride + jc] : T(0);
#pragma unroll
  for (int o = 0; o < NMAX; ++o) {
    if (o < t.nout) {
      T y = 0;
#pragma unroll
      for (int k = 0; k < NMAX; ++k) y += cf[o * NMAX + k] * x[k];
      const HPlane q = pl[t.nin + o];
      out[q.off + (int64_t)i * q.rowstride + jc] = y;
    }
  }
}

hipError_t launch_happly_planes(const HApplyLaunch& h, hipStream_t s);

hipError_t launch_happly(const HApplyLaunch& h, hipStream_t s) {
  if (h.cnt && h.nmax <= 16) return launch_happly_sparse(h, s);
  if (h.np > 0) return launch_happly_planes(h, s);
  if (h.nwork <= 0) return hipSuccess;
  if (h.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  dim3 grid((unsigned)h.nwork), block(256);
#define BST_HA(T_, N_)                                                                       \
  if (h.nmax == N_) {                                                                        \
    hipLaunchKernelGGL((happly_kernel<T_, N_>), grid, block, 0, s, h.tasks, h.planes, h.work, \
                       h.ptrs, reinterpret_cast<const T_*>(h.coef));                         \
    return hipGetLastError();                                                                \
  }
  if (h.t == ElemType::F64) {
    BST_HA(double, 8) BST_HA(double, 16) BST_HA(double, 32) BST_HA(double, 64)
  } else {
    BST_HA(float, 8) BST_HA(float, 16) BST_HA(float, 32) BST_HA(float, 64)
  }
#undef BST_HA
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------
// Lanczos vector kernels
// ------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sums acc[k] over the block in a fixed order and writes partial[k*G + blk].
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], int nv, double* red,
                                                   double* partial) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < nv) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) red[wave * NV + k] = v;
    }
  }
  __syncthreads();
  for (int k = tid; k < nv; k += 256) {
    const double v = ((red[k] + red[NV + k]) + red[2 * NV + k]) + red[3 * NV + k];
    partial[(int64_t)k * gridDim.x + blockIdx.x] = v;
  }
}

// sum_b partial[k*G + b] in a fixed order (thread-strided sums, wave sums,
// the four waves in order).  Called by all 256 threads of a block; every
// thread gets the sum.  red: 4 doubles of LDS.
__device__ __forceinline__ double block_sum_partials(const double* __restrict__ partial, int G, int k,
                                                     double* red) {
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < G; b += 256) s += partial[(int64_t)k * G + b];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  const double r = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return r;
}

// out[k] = sum_b partial[k*G + b]  (one block per k, fixed order)
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partial,
                                                              int G, double* __restrict__ out) {
  __shared__ double red[4];
  const double r = block_sum_partials(partial, G, blockIdx.x, red);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

static inline int vec_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

// Grid of the float32 basis pass: at most 512 blocks (two per CU at the
// pass's two waves per SIMD); its partial count is what the step kernel sums.
static inline int pass_grid_f32(int64_t n) {
  const int g = vec_grid((n + 1) / 2);
  return g < 512 ? g : 512;
}
// The float64 pass: 1024 workgroups (two rounds of resident workgroups at
// 40 rows: 205 VGPRs, two waves per SIMD); 512, one round, measured 7%
// slower on the 40-step chi = 4096 solve.
static inline int pass_grid_f64(int64_t n) { return vec_grid(n); }

// The Krylov basis is read through one base pointer plus a 32-bit per-lane
// byte offset (V is below 4 GiB, checked on the host), so the row addresses
// need neither 64-bit VGPR pairs nor one SGPR pair per row; the empty asm
// keeps the compiler from hoisting one offset per row into registers.
// Streaming loads and stores are non-temporal (V is read once per pass),
// except the one-pass schedule's store of the new residual row, which goes
// through the caches: the next operator application splits that row at once
// (0.81 -> 0.74 ms of split per 40-step chi = 4096 solve).
template <int NV>
__global__ __launch_bounds__(256) void multidot_kernel(const double* __restrict__ V, uint32_t ldv,
                                                       uint32_t n, int nv,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ partial) {
  // two elements per lane (16-byte loads; V rows and w are 16-byte aligned)
  __shared__ double red[4 * NV];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const char* Vb = reinterpret_cast<const char*>(V);
  const uint32_t rowb = ldv * 8u;
  const uint32_t stride = gridDim.x * 512u;
  typedef double dbl2 __attribute__((ext_vector_type(2)));
  for (uint32_t i = (blockIdx.x * 256u + threadIdx.x) * 2u; i + 1 < n; i += stride) {
    const dbl2 wi = *reinterpret_cast<const dbl2*>(w + i);
    uint32_t off = i * 8u;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if (k < nv) {
        const dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(Vb + off));
        acc[k] += v.x * wi.x + v.y * wi.y;
      }
      off += rowb;
      asm volatile("" : "+v"(off));
    }
  }
  if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t i = n - 1;
    for (int k = 0; k < NV; ++k)
      if (k < nv) acc[k] += V[(size_t)k * ldv + i] * w[i];
  }
  block_reduce_store<NV>(acc, nv, red, partial);
}

template <int NV>
__global__ __launch_bounds__(256) void project_kernel(const double* __restrict__ V, uint32_t ldv,
                                                      uint32_t n, int nv,
                                                      const double* __restrict__ c,
                                                      const double* w, double* wout, int mode,
                                                      double* __restrict__ partial) {
  __shared__ double red[4 * NV];
  __shared__ double cs[NV];
  for (int k = threadIdx.x; k < NV; k += 256) cs[k] = (k < nv) ? c[k] : 0.0;
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const char* Vb = reinterpret_cast<const char*>(V);
  const uint32_t rowb = ldv * 8u;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += stride) {
    double v[NV];
    double s = __builtin_nontemporal_load(w + i);
    uint32_t off = i * 8u;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      v[k] = (k < nv) ? __builtin_nontemporal_load(reinterpret_cast<const double*>(Vb + off)) : 0.0;
      off += rowb;
      asm volatile("" : "+v"(off));
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) s -= v[k] * cs[k];
    __builtin_nontemporal_store(s, wout + i);
    if (mode == 1) {
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] += v[k] * s;
    } else {
      acc[0] += s * s;
    }
  }
  block_reduce_store<NV>(acc, mode == 1 ? nv : 1, red, partial);
}

#define BST_NV_DISPATCH(KERNEL, ...)                                                      \
  do {                                                                                    \
    if (nv <= 8) hipLaunchKernelGGL((KERNEL<8>), __VA_ARGS__);                            \
    else if (nv <= 16) hipLaunchKernelGGL((KERNEL<16>), __VA_ARGS__);                     \
    else if (nv <= 24) hipLaunchKernelGGL((KERNEL<24>), __VA_ARGS__);                     \
    else if (nv <= 32) hipLaunchKernelGGL((KERNEL<32>), __VA_ARGS__);                     \
    else if (nv <= 40) hipLaunchKernelGGL((KERNEL<40>), __VA_ARGS__);                     \
    else if (nv <= 48) hipLaunchKernelGGL((KERNEL<48>), __VA_ARGS__);                     \
    else if (nv <= 64) hipLaunchKernelGGL((KERNEL<64>), __VA_ARGS__);                     \
    else if (nv <= 96) hipLaunchKernelGGL((KERNEL<96>), __VA_ARGS__);                     \
    else hipLaunchKernelGGL((KERNEL<128>), __VA_ARGS__);                                  \
  } while (0)

static bool fits32(const double* V, int64_t ldv, int64_t n, int nv) {
  (void)V;
  return n <= 0x7FFFFFFF && ldv <= 0x7FFFFFFF && (uint64_t)ldv * (uint64_t)nv * 8u < 0xFFFFFFFFull;
}

hipError_t launch_multidot(const double* V, int64_t ldv, int64_t n, int nv, const double* w,
                           double* partial, double* out, hipStream_t s) {
  if (nv < 1 || nv > kMaxVecs || !fits32(V, ldv, n, nv)) return hipErrorInvalidValue;
  const int G = vec_grid(n);
  BST_NV_DISPATCH(multidot_kernel, dim3(G), dim3(256), 0, s, V, (uint32_t)ldv, (uint32_t)n, nv, w,
                  partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(nv), dim3(256), 0, s, partial, G, out);
  return hipGetLastError();
}

hipError_t launch_project(const double* V, int64_t ldv, int64_t n, int nv, const double* c,
                          const double* w, double* wout, int mode, double* partial, double* out,
                          hipStream_t s) {
  if (nv < 1 || nv > kMaxVecs || !fits32(V, ldv, n, nv)) return hipErrorInvalidValue;
  const int G = vec_grid(n);
  BST_NV_DISPATCH(project_kernel, dim3(G), dim3(256), 0, s, V, (uint32_t)ldv, (uint32_t)n, nv, c,
                  w, wout, mode, partial);
  if (out)
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(mode == 1 ? nv : 1), dim3(256), 0, s, partial,
                       G, out);
  return hipGetLastError();
}

// End of a Lanczos step: every block adds the pass-3 partial norms in the
// same fixed order (so all blocks hold the same |w|^2), block 0 records
// alpha_j = c_j + d_j and beta_j = |w|, and the blocks write
// v_{j+1} = w / beta_j (skipped on the last step, vnext == nullptr).
__global__ __launch_bounds__(256) void lanczos_step_end_kernel(
    const double* __restrict__ partial, int G, const double* __restrict__ c,
    const double* __restrict__ d, int j, double* __restrict__ alpha, double* __restrict__ beta,
    double* __restrict__ norm2_out, const double* __restrict__ w, double* __restrict__ vnext,
    int64_t n) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < G; b += 256) s += partial[b];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  const double q = ((red[0] + red[1]) + red[2]) + red[3];
  if (blockIdx.x == 0 && tid == 0) {
    alpha[j] = c[j] + d[j];
    beta[j] = sqrt(q > 0.0 ? q : 0.0);
    norm2_out[0] = q;
  }
  if (!vnext) return;
  const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += stride) vnext[i] = w[i] * f;
}

hipError_t launch_lanczos_step_end(const double* partial, int64_t n_for_grid, const double* c,
                                   const double* d, int j, double* alpha, double* beta,
                                   double* norm2_out, const double* w, double* vnext, int64_t n,
                                   hipStream_t s) {
  const int G = vec_grid(n_for_grid);
  hipLaunchKernelGGL(lanczos_step_end_kernel, dim3(vnext ? vec_grid(n) : 1), dim3(256), 0, s,
                     partial, G, c, d, j, alpha, beta, norm2_out, w, vnext, n);
  return hipGetLastError();
}

// One pass over the Krylov basis per Lanczos step.  Row m of V holds u_m,
// the residual of step m-1 before its full projection (u_0 = v_0, the
// normalised start vector), and is never rewritten: the orthonormal vectors
// are v_k = sum_{m<=k} C[k][m] u_m with C lower triangular, one row per step
// (C[0][0] = 1).  At step j, dprev = V_{j-1}^T u_j (from the previous
// pass's sums u_m.u_j through C) and beta_{j-1} = |u_j - V_{j-1} dprev|, so
// v_j = (u_j - V_{j-1} dprev) / beta_{j-1}, which is row j of C:
//   C[j][m] = rb (delta_jm - sum_{k<j} dprev_k C[k][m]),  rb = 1 / beta_{j-1}.
// The operator was applied to u_j (z = H u_j); H v_j = (z - H V_{j-1} dprev)
// rb, and by the Lanczos relation H V_{j-1} = V_j T (T the tridiagonal of
// alpha, beta so far) the correction is the combination V_j e, e = T dprev.
// The three-term residual
//   w = H v_j - a v_j - beta_{j-1} v_{j-1}
// (a = v_j.H v_j from g = u_j.z and the same relation) is then measured
// against all of u_0..u_j in the same pass; its projection onto V_j is
// applied lagged, in the next step.  This is the delayed-reorthogonalisation
// idea of low-synchronisation Gram-Schmidt (Swirydowicz et al., Numer.
// Linear Algebra Appl. 2021; Bielich et al., Parallel Comput. 2022)
// specialised to the symmetric three-term recurrence; in exact arithmetic
// alpha_j and beta_j equal those of Lanczos with two full classical
// Gram-Schmidt passes.  Keeping the rows as written (C carries the
// projections and scalings) leaves the pass one store per element, w.
//
// The scalars of step j from g = u_j.z (al, be, dp hold alpha, beta, dprev
// for k < j):
//   v_j . z = rb (g - dprev . f),  f = (T^T y)_{k<j},  y = (dprev, beta_{j-1});
//   e = T dprev over rows 0..j;  coef_k = rb e_k (+ beta_{j-1} for k = j-1),
// the coefficients of v_0..v_j in w = z rb - sum_k coef_k v_k; and aest, the
// three-term estimate of alpha_j.  In the rows as stored,
//   w = z rb - sum_{m<=j} cp_m u_m,  cp_m = sum_{k=m..j} coef_k C[k][m].
// lanczos_step_scalars_kernel evaluates them.

// The pass of step j: per element
//   w = z rb - sum_{m<=j} cp_m u_m      written to vnext (if any)
// and the block partials of u_m.w (m <= j) and w.w (j + 2 values).
// z is float64, or float32 when the matvec's float32 accumulators wrote it
// (exact: the same values).
template <int NV, typename TZ>
__global__ __launch_bounds__(256) void lanczos_pass_kernel(
    const double* V, uint32_t ldv, uint32_t n, int j, const TZ* __restrict__ z,
    const double* __restrict__ coef, const double* __restrict__ beta, double* vnext,
    double* __restrict__ partial) {
  constexpr int NR = NV + 2;
  __shared__ double red[4 * NR];
  __shared__ double cs[NV];
  const int tid = threadIdx.x;
  const double b = j > 0 ? beta[j - 1] : 1.0;
  const double rb = b > 0.0 ? 1.0 / b : 0.0;
  for (int k = tid; k < NV; k += 256) cs[k] = k <= j ? coef[k] : 0.0;
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  double accw = 0.0;
  const char* Vb = reinterpret_cast<const char*>(V);
  const uint32_t rowb = ldv * 8u;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t i = blockIdx.x * 256u + tid; i < n; i += stride) {
    double v[NV];
    uint32_t off = i * 8u;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      v[k] = (k <= j) ? __builtin_nontemporal_load(reinterpret_cast<const double*>(Vb + off)) : 0.0;
      off += rowb;
      asm volatile("" : "+v"(off));
    }
    const double zi = (double)__builtin_nontemporal_load(z + i);
    double sacc = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) sacc += cs[k] * v[k];
    const double w = zi * rb - sacc;
    if (vnext) vnext[i] = w;
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += v[k] * w;
    accw += w * w;
  }
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k <= j) {
      const double r = wave_sum(acc[k]);
      if (lane == 0) red[wave * NR + k] = r;
    }
  }
  {
    const double r2 = wave_sum(accw);
    if (lane == 0) red[wave * NR + j + 1] = r2;
  }
  __syncthreads();
  for (int k = tid; k < j + 2; k += 256) {
    const double r = ((red[k] + red[NR + k]) + red[2 * NR + k]) + red[3 * NR + k];
    partial[(int64_t)k * gridDim.x + blockIdx.x] = r;
  }
}

// The same pass over a float32 basis (the split forms; z float32 too): two
// elements per lane, so every row access is 8 bytes.  w is rounded to
// float32 before it enters the dot products, so the measured projections
// are those of the rows as stored.  An odd n leaves one padding element in
// the last pair (rows are padded, z holds n doubles): it is read, never
// counted.
template <int NV, typename TZ>
__global__ __launch_bounds__(256) void lanczos_pass_f32_kernel(
    const float* V, uint32_t ldv, uint32_t n, int j, const TZ* __restrict__ z,
    const double* __restrict__ coef, const double* __restrict__ beta, float* vnext,
    double* __restrict__ partial) {
  typedef float fl2 __attribute__((ext_vector_type(2)));
  constexpr int NR = NV + 2;
  __shared__ double red[4 * NR];
  __shared__ double cs[NV];
  const int tid = threadIdx.x;
  const double b = j > 0 ? beta[j - 1] : 1.0;
  const double rb = b > 0.0 ? 1.0 / b : 0.0;
  for (int k = tid; k < NV; k += 256) cs[k] = k <= j ? coef[k] : 0.0;
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  double accw = 0.0;
  const char* Vb = reinterpret_cast<const char*>(V);
  const uint32_t rowb = ldv * 4u;
  const uint32_t npair = (n + 1u) / 2u;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t p = blockIdx.x * 256u + tid; p < npair; p += stride) {
    const bool two = 2u * p + 1u < n;
    fl2 v[NV];
    uint32_t off = p * 8u;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      v[k] = (k <= j) ? __builtin_nontemporal_load(reinterpret_cast<const fl2*>(Vb + off)) : fl2{0.f, 0.f};
      if (!two) v[k].y = 0.f;
      off += rowb;
      asm volatile("" : "+v"(off));
    }
    double z0, z1;
    if constexpr (sizeof(TZ) == 4) {
      if (two) {
        const fl2 zz = __builtin_nontemporal_load(reinterpret_cast<const fl2*>(z) + p);
        z0 = zz.x;
        z1 = zz.y;
      } else {
        z0 = __builtin_nontemporal_load(z + 2u * p);
        z1 = 0.0;
      }
    } else {
      z0 = __builtin_nontemporal_load(z + 2u * p);
      z1 = two ? __builtin_nontemporal_load(z + 2u * p + 1u) : 0.0;
    }
    // Register budget (two waves per SIMD): the coefficients are read from
    // LDS eight rows at a time, and the float64 images of the rows are formed
    // again for the dot products instead of being kept from this loop.
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      s0 += cs[k] * v[k].x;
      s1 += cs[k] * v[k].y;
      if (k % 8 == 7) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) asm volatile("" : "+v"(v[k]));
    const float w0 = (float)(z0 * rb - s0);
    const float w1 = two ? (float)(z1 * rb - s1) : 0.f;
    if (vnext) __builtin_nontemporal_store(fl2{w0, w1}, reinterpret_cast<fl2*>(vnext) + p);
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += (double)v[k].x * w0 + (double)v[k].y * w1;
    accw += (double)w0 * w0 + (double)w1 * w1;
  }
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k <= j) {
      const double r = wave_sum(acc[k]);
      if (lane == 0) red[wave * NR + k] = r;
    }
  }
  {
    const double r2 = wave_sum(accw);
    if (lane == 0) red[wave * NR + j + 1] = r2;
  }
  __syncthreads();
  for (int k = tid; k < j + 2; k += 256) {
    const double r = ((red[k] + red[NR + k]) + red[2 * NR + k]) + red[3 * NR + k];
    partial[(int64_t)k * gridDim.x + blockIdx.x] = r;
  }
}

// End of step j: dn = (V_j^T w, w.w).  alpha_j = aest + dn_j (the lagged
// projection's share along v_j); beta_j^2 = w.w - |dn|^2 (the norm of w once
// projected); dprev <- dn.
// alpha_j and beta_j from ds = dn (one thread).
__device__ __forceinline__ void step_end(const double* ds, double aest, int j, double& alpha_j,
                                         double& beta_j) {
  double ss = 0.0;
  for (int k = 0; k <= j; ++k) ss += ds[k] * ds[k];
  const double q = ds[j + 1] - ss;
  alpha_j = aest + ds[j];
  beta_j = sqrt(q > 0.0 ? q : 0.0);
}

// The basis pass measures w against the rows as stored (u_m . w); the
// projections onto the orthonormal vectors are v_k . w = sum_{m<=k} C[k][m]
// (u_m . w).  Rows k < nk of C (row k at cmat + k * kMaxVecs) are spread
// over the 16 waves of a 1024-thread block, row k on wave k % 16, columns
// lane and lane + 64; each wave loads its rows once, at the start.
constexpr int kCRowsPerWave = kMaxVecs / 16;
__device__ __forceinline__ void load_c_rows(const double* __restrict__ cmat, int nk, int wave, int lane,
                                            double (&creg)[kCRowsPerWave][2]) {
#pragma unroll
  for (int r = 0; r < kCRowsPerWave; ++r) {
    const int k = wave + 16 * r;
    creg[r][0] = (k < nk && lane <= k) ? cmat[(int64_t)k * kMaxVecs + lane] : 0.0;
    creg[r][1] = (k < nk && lane + 64 <= k) ? cmat[(int64_t)k * kMaxVecs + lane + 64] : 0.0;
  }
}
// out[k] = sum_{m<=k} C[k][m] x[m] for k < nk (x in LDS, valid below nk);
// each row's sum is a wave_sum in a fixed order.
__device__ __forceinline__ void c_times(const double (&creg)[kCRowsPerWave][2], int nk, int wave, int lane,
                                        const double* x, double* out) {
#pragma unroll
  for (int r = 0; r < kCRowsPerWave; ++r) {
    const int k = wave + 16 * r;
    if (k < nk) {
      const double x0 = lane <= k ? x[lane] : 0.0;
      const double x1 = lane + 64 <= k ? x[lane + 64] : 0.0;
      const double t = wave_sum(creg[r][0] * x0 + creg[r][1] * x1);
      if (lane == 0) out[k] = t;
    }
  }
}
// Per-wave partials of sum_{k<nk} y[k] C[k][m] over the wave's rows, for
// m = lane, lane + 64, into part[wave][m].
__device__ __forceinline__ void ct_times_part(const double (&creg)[kCRowsPerWave][2], int nk, int wave,
                                              int lane, const double* y, double (*part)[kMaxVecs]) {
  double p0 = 0.0, p1 = 0.0;
#pragma unroll
  for (int r = 0; r < kCRowsPerWave; ++r) {
    const int k = wave + 16 * r;
    if (k < nk) {
      p0 += y[k] * creg[r][0];
      p1 += y[k] * creg[r][1];
    }
  }
  part[wave][lane] = p0;
  part[wave][lane + 64] = p1;
}

// End of the last step j: the raw sums dn (u_m . w for m <= j, then w.w)
// become dprev = V_j^T w through C, then alpha_j, beta_j as step_end.
__global__ __launch_bounds__(1024) void lanczos_end_kernel(const double* __restrict__ dn,
                                                           const double* __restrict__ aest, int j,
                                                           const double* __restrict__ cmat,
                                                           double* __restrict__ dprev,
                                                           double* __restrict__ alpha,
                                                           double* __restrict__ beta) {
  __shared__ double raw[kMaxVecs + 2], ds[kMaxVecs + 2];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double creg[kCRowsPerWave][2];
  load_c_rows(cmat, j + 1, wave, lane, creg);
  for (int k = tid; k < j + 2; k += 1024) raw[k] = dn[k];
  __syncthreads();
  c_times(creg, j + 1, wave, lane, raw, ds);
  if (tid == 0) ds[j + 1] = raw[j + 1];
  __syncthreads();
  for (int k = tid; k <= j; k += 1024) dprev[k] = ds[k];
  if (tid != 0) return;
  step_end(ds, aest[0], j, alpha[j], beta[j]);
}

// The scalar work between two basis passes, in one block of 1024 threads:
// the sums of the u_j.z, z.z partials of dot2_kernel (g) beside the sums of
// the pass of step pj that dot2_kernel already left in dn (u_m . u_j for
// m <= pj, then u_j . u_j), which C turns into dprev = V_pj^T u_j; then the
// end of step pj (alpha, beta as lanczos_end_kernel), row j of C, and the
// scalars of step j, first as coefficients of v_0..v_j, then of the rows as
// stored (coef).  One wave forms each partial sum (lane l adds partials l,
// l + 64, ..., then the wave sum); every load of a sum is issued at once
// (grids of at most 1024 blocks).  The scalars themselves take one wave,
// lane-parallel over k.  pj < 0: no pass before (step 0).
__global__ __launch_bounds__(1024) void lanczos_step_scalars_kernel(
    int pj, const double* __restrict__ dpart, int dG, int j, double* __restrict__ dn,
    double* __restrict__ g, double* __restrict__ alpha, double* __restrict__ beta,
    double* __restrict__ dprev, double* __restrict__ coef, double* __restrict__ aest,
    double* __restrict__ cmat) {
  __shared__ double sv[kMaxVecs + 4], dps[kMaxVecs];
  __shared__ double al[kMaxVecs], be[kMaxVecs];
  __shared__ double cf[kMaxVecs], crow[1];
  __shared__ double part[16][kMaxVecs], part2[16][kMaxVecs];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int npv = pj >= 0 ? pj + 2 : 0;
  double creg[kCRowsPerWave][2];
  load_c_rows(cmat, j, wave, lane, creg);   // rows 0..j-1
  // sv[0..npv): the previous pass's sums, formed by dot2_kernel into dn
  for (int k = tid; k < npv; k += 1024) sv[k] = dn[k];
  // sv[npv], sv[npv + 1]: u_j.z and z.z, one wave each (lane l adds
  // partials l, l + 64, ..., then the wave sum)
  if (wave < 2) {
    const double* __restrict__ src = dpart + (int64_t)wave * dG;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = lane + 64 * i < dG ? src[lane + 64 * i] : 0.0;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += x[i];
    t = wave_sum(t);
    if (lane == 0) sv[npv + wave] = t;
  }
  for (int k = tid; k < pj; k += 1024) {
    al[k] = alpha[k];
    be[k] = beta[k];
  }
  __syncthreads();
  // dprev_k = v_k . u_j = sum_{m<=k} C[k][m] (u_m . u_j), k < j
  c_times(creg, j, wave, lane, sv, dps);
  __syncthreads();
  // dps = dprev, sv[j] = u_j . u_j, sv[npv] = u_j.z, sv[npv + 1] = z.z;
  // part = per-wave shares of dprev^T C (row j of C: rb (e_j - C^T dprev))
  for (int k = tid; k < j; k += 1024) dprev[k] = dps[k];
  ct_times_part(creg, j, wave, lane, dps, part);
  if (wave == 0) {
    // The scalars in wave 0, lane-parallel over the step index k (k <
    // kMaxVecs, two per lane).  Each sum is a wave_sum in a fixed order
    // whose result lane 0 broadcasts, so every lane continues with the same
    // value.
    // End of step pj (as step_end): alpha_pj, beta_pj.
    const double* dp = dps;
    double apj = 0.0, bpj = 0.0;
    if (pj >= 0) {
      double t = 0.0;
      for (int k = lane; k <= pj; k += 64) t += dp[k] * dp[k];
      const double ss = __shfl(wave_sum(t), 0, 64);
      const double q = sv[pj + 1] - ss;
      apj = aest[0] + dp[pj];
      bpj = sqrt(q > 0.0 ? q : 0.0);
      if (lane == 0) {
        alpha[pj] = apj;
        beta[pj] = bpj;
      }
    }
    if (lane == 0) {
      g[0] = sv[npv];
      g[1] = sv[npv + 1];
    }
    auto AL = [&](int k) { return k == pj ? apj : al[k]; };
    auto BE = [&](int k) { return k == pj ? bpj : be[k]; };
    const double bp = j > 0 ? bpj : 1.0;
    const double rb = bp > 0.0 ? 1.0 / bp : 0.0;
    // Scalars of step j = pj + 1.
    double t = 0.0;
    for (int k = lane; k < j; k += 64) {
      const double yn = k + 1 < j ? dp[k + 1] : bp;
      double f = AL(k) * dp[k] + BE(k) * yn;
      if (k > 0) f += BE(k - 1) * dp[k - 1];
      t += dp[k] * f;
    }
    const double sdot = __shfl(wave_sum(t), 0, 64);
    const double vz = rb * (sv[npv] - sdot);
    for (int i = lane; i < j; i += 64) {
      double e = AL(i) * dp[i];
      if (i > 0) e += BE(i - 1) * dp[i - 1];
      if (i + 1 < j) e += BE(i) * dp[i + 1];
      cf[i] = rb * e + (i == j - 1 ? bp : 0.0);
    }
    if (lane == 0) {
      const double ej = j > 0 ? BE(j - 1) * dp[j - 1] : 0.0;
      const double a = rb * (vz - ej);
      cf[j] = rb * ej + a;
      aest[0] = a;
      crow[0] = rb;   // crow[0] carries rb to the other waves
    }
  }
  __syncthreads();
  // In the rows as stored, with C[j][m] = rb (delta_jm - (C^T dprev)_m):
  //   coef_m = sum_{k<j} (cf_k - cf_j rb dprev_k) C[k][m] + cf_j rb delta_jm;
  // the waves' shares of the sum go to part2, then one thread per m adds
  // them in wave order and also stores row j of C.
  const double rb = crow[0];
  {
    const double cj = cf[j] * rb;
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int r = 0; r < kCRowsPerWave; ++r) {
      const int k = wave + 16 * r;
      if (k < j) {
        const double y = cf[k] - cj * dps[k];
        p0 += y * creg[r][0];
        p1 += y * creg[r][1];
      }
    }
    part2[wave][lane] = p0;
    part2[wave][lane + 64] = p1;
  }
  __syncthreads();
  for (int m = tid; m <= j; m += 1024) {
    double cs = 0.0, cp = 0.0;
    for (int w = 0; w < 16; ++w) {
      cs += part[w][m];
      cp += part2[w][m];
    }
    const double dj = m == j ? 1.0 : 0.0;
    cmat[(int64_t)j * kMaxVecs + m] = rb * (dj - cs);
    coef[m] = cp + cf[j] * rb * dj;
  }
}

template <typename TZ>
static hipError_t pass_f64_impl(const double* V, int64_t ldv, int64_t n, int j, const TZ* z,
                                const double* coef, const double* beta, double* vnext, double* partial,
                                double* dn, hipStream_t s) {
  if (j < 0 || j + 2 > kMaxVecs + 1 || !fits32(V, ldv, n, j + 1)) return hipErrorInvalidValue;
  const int G = pass_grid_f64(n);
  const int nv = j + 1;   // rows 0..j
#define BST_PF64(NV_)                                                                                  \
  hipLaunchKernelGGL((lanczos_pass_kernel<NV_, TZ>), dim3(G), dim3(256), 0, s, V, (uint32_t)ldv, \
                     (uint32_t)n, j, z, coef, beta, vnext, partial)
  if (nv <= 8) BST_PF64(8);
  else if (nv <= 16) BST_PF64(16);
  else if (nv <= 24) BST_PF64(24);
  else if (nv <= 32) BST_PF64(32);
  else if (nv <= 40) BST_PF64(40);
  else if (nv <= 48) BST_PF64(48);
  else if (nv <= 64) BST_PF64(64);
  else if (nv <= 96) BST_PF64(96);
  else BST_PF64(128);
#undef BST_PF64
  if (dn) hipLaunchKernelGGL(reduce_partials_kernel, dim3(j + 2), dim3(256), 0, s, partial, G, dn);
  return hipGetLastError();
}
hipError_t launch_lanczos_pass(const double* V, int64_t ldv, int64_t n, int j, const double* z,
                               const double* coef, const double* beta, double* vnext, double* partial,
                               double* dn, hipStream_t s) {
  return pass_f64_impl(V, ldv, n, j, z, coef, beta, vnext, partial, dn, s);
}
hipError_t launch_lanczos_pass(const double* V, int64_t ldv, int64_t n, int j, const float* z,
                               const double* coef, const double* beta, double* vnext, double* partial,
                               double* dn, hipStream_t s) {
  return pass_f64_impl(V, ldv, n, j, z, coef, beta, vnext, partial, dn, s);
}

hipError_t launch_lanczos_pass(const float* V, int64_t ldv, int64_t n, int j, const float* z,
                               const double* coef, const double* beta, float* vnext, double* partial,
                               double* dn, hipStream_t s) {
  if (j < 0 || j + 2 > kMaxVecs + 1 || n > 0x7FFFFFFF || ldv > 0x7FFFFFFF || ldv % 2 ||
      (uint64_t)ldv * (uint64_t)(j + 1) * 4u >= 0xFFFFFFFFull)
    return hipErrorInvalidValue;
  const int G = pass_grid_f32(n);
  const int nv = j + 1;   // rows 0..j
  #define BST_PF32(NV_)                                                                                      \
  hipLaunchKernelGGL((lanczos_pass_f32_kernel<NV_, float>), dim3(G), dim3(256), 0, s, V, (uint32_t)ldv, \
                     (uint32_t)n, j, z, coef, beta, vnext, partial)
  if (nv <= 8) BST_PF32(8);
  else if (nv <= 16) BST_PF32(16);
  else if (nv <= 24) BST_PF32(24);
  else if (nv <= 32) BST_PF32(32);
  else if (nv <= 40) BST_PF32(40);
  else if (nv <= 48) BST_PF32(48);
  else if (nv <= 64) BST_PF32(64);
  else if (nv <= 96) BST_PF32(96);
  else BST_PF32(128);
#undef BST_PF32
  if (dn) hipLaunchKernelGGL(reduce_partials_kernel, dim3(j + 2), dim3(256), 0, s, partial, G, dn);
  return hipGetLastError();
}

hipError_t launch_lanczos_pass_sums(int64_t n, int j, bool f32, const double* partial, double* dn,
                                   hipStream_t s) {
  if (j < 0 || j + 2 > kMaxVecs + 1 || n < 0) return hipErrorInvalidValue;
  const int G = f32 ? pass_grid_f32(n) : pass_grid_f64(n);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(j + 2), dim3(256), 0, s, partial, G, dn);
  return hipGetLastError();
}

hipError_t launch_lanczos_end(const double* dn, const double* aest, int j, const double* cmat,
                              double* dprev, double* alpha, double* beta, hipStream_t s) {
  if (j < 0 || j >= kMaxVecs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lanczos_end_kernel, dim3(1), dim3(1024), 0, s, dn, aest, j, cmat, dprev, alpha, beta);
  return hipGetLastError();
}

// y = sum_{k<nv} coef_k V_k (the Ritz vector).  Two elements per lane, one
// 8- or 16-byte load per basis row, 32-bit byte offsets (the launcher checks
// that nv rows fit); rows are padded to an even length, so the second element
// of the last pair is inside the row even when n is odd (it is not stored).
template <int NV, typename TV>
__global__ __launch_bounds__(256) void combine_kernel(const TV* __restrict__ V, uint32_t ldv,
                                                      uint32_t n, int nv,
                                                      const double* __restrict__ coef,
                                                      double* __restrict__ y) {
  typedef TV tv2 __attribute__((ext_vector_type(2)));
  __shared__ double cs[NV];
  for (int k = threadIdx.x; k < NV; k += 256) cs[k] = (k < nv) ? coef[k] : 0.0;
  __syncthreads();
  const char* Vb = reinterpret_cast<const char*>(V);
  const uint32_t rowb = ldv * (uint32_t)sizeof(TV);
  const uint32_t npair = (n + 1u) / 2u;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < npair; p += stride) {
    tv2 v[NV];
    uint32_t off = p * (uint32_t)sizeof(tv2);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      v[k] = (k < nv) ? __builtin_nontemporal_load(reinterpret_cast<const tv2*>(Vb + off)) : tv2{0, 0};
      off += rowb;
      asm volatile("" : "+v"(off));
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      s0 += cs[k] * (double)v[k].x;
      s1 += cs[k] * (double)v[k].y;
      if (k % 8 == 7) __builtin_amdgcn_sched_barrier(0);
    }
    y[2u * p] = s0;
    if (2u * p + 1u < n) y[2u * p + 1u] = s1;
  }
}

template <typename TV>
static hipError_t combine_impl(const TV* V, int64_t ldv, int64_t n, int nv, const double* coef, double* y,
                               hipStream_t s) {
  if (nv < 1 || nv > kMaxVecs || n > 0x7FFFFFFF || ldv > 0x7FFFFFFF || ldv % 2 || ldv < n ||
      (uint64_t)ldv * (uint64_t)nv * sizeof(TV) >= 0xFFFFFFFFull)
    return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const int G = vec_grid((n + 1) / 2);
#define BST_CMB(NV_) \
  hipLaunchKernelGGL((combine_kernel<NV_, TV>), dim3(G), dim3(256), 0, s, V, (uint32_t)ldv, (uint32_t)n, nv, coef, y)
  if (nv <= 8) BST_CMB(8);
  else if (nv <= 16) BST_CMB(16);
  else if (nv <= 24) BST_CMB(24);
  else if (nv <= 32) BST_CMB(32);
  else if (nv <= 40) BST_CMB(40);
  else if (nv <= 48) BST_CMB(48);
  else if (nv <= 64) BST_CMB(64);
  else if (nv <= 96) BST_CMB(96);
  else BST_CMB(128);
#undef BST_CMB
  return hipGetLastError();
}
hipError_t launch_combine(const double* V, int64_t ldv, int64_t n, int nv, const double* coef,
                          double* y, hipStream_t s) {
  return combine_impl(V, ldv, n, nv, coef, y, s);
}
hipError_t launch_combine(const float* V, int64_t ldv, int64_t n, int nv, const double* coef,
                          double* y, hipStream_t s) {
  return combine_impl(V, ldv, n, nv, coef, y, s);
}

template <typename TD>
__global__ __launch_bounds__(256) void scale_rnorm_kernel(const double* __restrict__ src,
                                                          const double* __restrict__ norm2,
                                                          TD* __restrict__ dst, int64_t n) {
  const double q = norm2[0];
  const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = (TD)(src[i] * f);
}

hipError_t launch_scale_rnorm(const double* src, const double* norm2, double* dst, int64_t n,
                              hipStream_t s) {
  hipLaunchKernelGGL(scale_rnorm_kernel<double>, dim3(vec_grid(n)), dim3(256), 0, s, src, norm2, dst, n);
  return hipGetLastError();
}
hipError_t launch_scale_rnorm(const double* src, const double* norm2, float* dst, int64_t n,
                              hipStream_t s) {
  hipLaunchKernelGGL(scale_rnorm_kernel<float>, dim3(vec_grid(n)), dim3(256), 0, s, src, norm2, dst, n);
  return hipGetLastError();
}

// PAIR (x and y of one type, aligned to two elements, n < 2^31): two
// elements per lane with one 8-byte (float32) or 16-byte (float64) load
// each; otherwise one element per lane.
template <typename TX, typename TY, bool PAIR>
__global__ __launch_bounds__(256) void dot2_kernel(const TX* __restrict__ x,
                                                   const TY* __restrict__ y, int64_t n,
                                                   double* __restrict__ partial,
                                                   const double* __restrict__ ppart = nullptr,
                                                   int pG = 0, int npv = 0,
                                                   double* __restrict__ psum = nullptr) {
  __shared__ double red[4 * 2];
  // Inside a Lanczos step: wave 0 of workgroup v (v < npv) also sums row v
  // of the previous basis pass's partials (pG <= 1024 per row) into psum[v],
  // in the step scalars kernel's order (lane l adds entries l, l + 64, ...,
  // then the wave sum), so that kernel reads npv finished sums.
  if (npv > 0 && threadIdx.x < 64) {
    const int lane = threadIdx.x;
    for (int v = blockIdx.x; v < npv; v += gridDim.x) {
      const double* __restrict__ src = ppart + (int64_t)v * pG;
      double xs[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) xs[i] = lane + 64 * i < pG ? src[lane + 64 * i] : 0.0;
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) t += xs[i];
      t = wave_sum(t);
      if (lane == 0) psum[v] = t;
    }
  }
  double acc[2] = {0.0, 0.0};
  if constexpr (PAIR && sizeof(TX) == 4 && sizeof(TY) == 4) {
    typedef float fl2 __attribute__((ext_vector_type(2)));
    const uint32_t npair = (uint32_t)((n + 1) / 2);
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < npair; p += stride) {
      fl2 xv, yv;
      if (2u * p + 1u < (uint32_t)n) {
        xv = __builtin_nontemporal_load(reinterpret_cast<const fl2*>(x) + p);
        yv = __builtin_nontemporal_load(reinterpret_cast<const fl2*>(y) + p);
      } else {
        xv = fl2{x[2u * p], 0.f};
        yv = fl2{y[2u * p], 0.f};
      }
      acc[0] += (double)xv.x * (double)yv.x;
      acc[0] += (double)xv.y * (double)yv.y;
      acc[1] += (double)yv.x * (double)yv.x;
      acc[1] += (double)yv.y * (double)yv.y;
    }
  } else if constexpr (PAIR && sizeof(TX) == 8 && sizeof(TY) == 4) {
    // float64 x (16-byte aligned), float32 y (8-byte aligned): the pairs
    // and the order of the float64 pair path, y widened exactly
    typedef float fl2 __attribute__((ext_vector_type(2)));
    const int64_t npair = (n + 1) / 2;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npair; p += stride) {
      dbl2v xv, yv;
      if (2 * p + 1 < n) {
        xv = __builtin_nontemporal_load(reinterpret_cast<const dbl2v*>(x) + p);
        const fl2 yf = __builtin_nontemporal_load(reinterpret_cast<const fl2*>(y) + p);
        yv = dbl2v{(double)yf.x, (double)yf.y};
      } else {
        xv = dbl2v{(double)x[2 * p], 0.0};
        yv = dbl2v{(double)y[2 * p], 0.0};
      }
      acc[0] += xv.x * yv.x;
      acc[0] += xv.y * yv.y;
      acc[1] += yv.x * yv.x;
      acc[1] += yv.y * yv.y;
    }
  } else if constexpr (PAIR && sizeof(TX) == 8 && sizeof(TY) == 8) {
    // float64 x and y, both 16-byte aligned: two elements per 16-byte load
    const int64_t npair = (n + 1) / 2;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npair; p += stride) {
      dbl2v xv, yv;
      if (2 * p + 1 < n) {
        xv = __builtin_nontemporal_load(reinterpret_cast<const dbl2v*>(x) + p);
        yv = __builtin_nontemporal_load(reinterpret_cast<const dbl2v*>(y) + p);
      } else {
        xv = dbl2v{(double)x[2 * p], 0.0};
        yv = dbl2v{(double)y[2 * p], 0.0};
      }
      acc[0] += xv.x * yv.x;
      acc[0] += xv.y * yv.y;
      acc[1] += yv.x * yv.x;
      acc[1] += yv.y * yv.y;
    }
  } else {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
      const double yi = (double)y[i];
      acc[0] += (double)x[i] * yi;
      acc[1] += yi * yi;
    }
  }
  block_reduce_store<2>(acc, 2, red, partial);
}

template <typename TX>
static hipError_t dot2_impl(const TX* x, const double* y, int64_t n, double* partial, double* out,
                            hipStream_t s) {
  const int G = vec_grid(n);
  hipLaunchKernelGGL((dot2_kernel<TX, double, false>), dim3(G), dim3(256), 0, s, x, y, n, partial);
  if (out) hipLaunchKernelGGL(reduce_partials_kernel, dim3(2), dim3(256), 0, s, partial, G, out);
  return hipGetLastError();
}
hipError_t launch_dot2(const double* x, const double* y, int64_t n, double* partial, double* out,
                       hipStream_t s) {
  return dot2_impl(x, y, n, partial, out, s);
}
hipError_t launch_dot2(const float* x, const double* y, int64_t n, double* partial, double* out,
                       hipStream_t s) {
  return dot2_impl(x, y, n, partial, out, s);
}

template <typename TX, typename TZ>
static hipError_t dot_step_impl(const TX* x, const TZ* z, int64_t n, double* dpart,
                                const double* ppart, int pj, double* dn, int j, double* g,
                                double* alpha, double* beta, double* dprev, double* coef,
                                double* aest, double* cmat, hipStream_t s) {
  if (j < 0 || j >= kMaxVecs || pj != j - 1 || n < 0) return hipErrorInvalidValue;
  // two elements per lane: x and z each aligned to two of its elements (one
  // 8- or 16-byte load each)
  const bool aligned = (reinterpret_cast<uintptr_t>(x) & (2 * sizeof(TX) - 1)) == 0 &&
                       (reinterpret_cast<uintptr_t>(z) & (2 * sizeof(TZ) - 1)) == 0;
  const bool pair = sizeof(TX) >= sizeof(TZ) && n <= 0x7FFFFFFF && aligned;
  const int G = pair ? vec_grid((n + 1) / 2) : vec_grid(n);
  // the basis pass's grid: one element (float64 rows) or pair (float32) per lane
  const int pG = sizeof(TX) == 4 ? pass_grid_f32(n) : pass_grid_f64(n);
  if (G > 1024 || pG > 1024) return hipErrorInvalidValue;
  // the previous pass's sums go straight into dn (the scalars kernel reads them there)
  const int npv = pj >= 0 ? pj + 2 : 0;
  if (pair)
    hipLaunchKernelGGL((dot2_kernel<TX, TZ, true>), dim3(G), dim3(256), 0, s, x, z, n, dpart, ppart, pG, npv,
                       dn);
  else
    hipLaunchKernelGGL((dot2_kernel<TX, TZ, false>), dim3(G), dim3(256), 0, s, x, z, n, dpart, ppart, pG, npv,
                       dn);
  hipLaunchKernelGGL(lanczos_step_scalars_kernel, dim3(1), dim3(1024), 0, s, pj, dpart, G, j, dn, g, alpha,
                     beta, dprev, coef, aest, cmat);
  return hipGetLastError();
}
hipError_t launch_lanczos_dot_step(const double* x, const double* z, int64_t n, double* dpart,
                                   const double* ppart, int pj, double* dn, int j, double* g,
                                   double* alpha, double* beta, double* dprev, double* coef,
                                   double* aest, double* cmat, hipStream_t s) {
  return dot_step_impl(x, z, n, dpart, ppart, pj, dn, j, g, alpha, beta, dprev, coef, aest, cmat, s);
}
hipError_t launch_lanczos_dot_step(const double* x, const float* z, int64_t n, double* dpart,
                                   const double* ppart, int pj, double* dn, int j, double* g,
                                   double* alpha, double* beta, double* dprev, double* coef,
                                   double* aest, double* cmat, hipStream_t s) {
  return dot_step_impl(x, z, n, dpart, ppart, pj, dn, j, g, alpha, beta, dprev, coef, aest, cmat, s);
}
hipError_t launch_lanczos_dot_step(const float* x, const float* z, int64_t n, double* dpart,
                                   const double* ppart, int pj, double* dn, int j, double* g,
                                   double* alpha, double* beta, double* dprev, double* coef,
                                   double* aest, double* cmat, hipStream_t s) {
  return dot_step_impl(x, z, n, dpart, ppart, pj, dn, j, g, alpha, beta, dprev, coef, aest, cmat, s);
}

__global__ __launch_bounds__(256) void resid_kernel(const double* __restrict__ hy,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ num, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double red[4];
  const double e = num[0] / num[1];
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const double r = hy[i] - e * y[i];
    acc[0] += r * r;
  }
  block_reduce_store<1>(acc, 1, red, partial);
}

hipError_t launch_resid(const double* hy, const double* y, const double* num, int64_t n,
                        double* partial, double* out, hipStream_t s) {
  const int G = vec_grid(n);
  hipLaunchKernelGGL(resid_kernel, dim3(G), dim3(256), 0, s, hy, y, num, n, partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partial, G, out);
  return hipGetLastError();
}

// 480 pointers (3840 bytes) per launch: within the 4 KiB of kernel arguments
constexpr int kPtrChunk = 480;
struct PtrChunk {
  void* p[kPtrChunk];
};
__global__ __launch_bounds__(512) void set_ptrs_kernel(void** table, PtrChunk c, int n) {
  const int i = threadIdx.x;
  if (i < n) table[i] = c.p[i];
}

// Writes a device pointer table through a kernel argument (no host staging
// buffer has to outlive the call).
hipError_t launch_set_ptrs(void** table, void* const* src, int n, hipStream_t s) {
  for (int base = 0; base < n; base += kPtrChunk) {
    PtrChunk c{};
    const int m = n - base < kPtrChunk ? n - base : kPtrChunk;
    for (int i = 0; i < m; ++i) c.p[i] = src[base + i];
    hipLaunchKernelGGL(set_ptrs_kernel, dim3(1), dim3(512), 0, s, table + base, c, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


}  // namespace bst

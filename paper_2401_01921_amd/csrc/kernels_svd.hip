// Symmetric SVD kernels (Sec. "Singular value decomposition"): the block
// matrices of every charge sector are gathered into the tall orientation X,
// each sector's SVD runs as one-sided Jacobi (Hestenes) in one workgroup,
// the truncation is selected across all sectors by one workgroup, and the
// kept columns are written into the block layouts of U and V^dagger.
//
// One-sided Jacobi: for a pair of columns (x_i, x_j) with a = |x_i|^2,
// b = |x_j|^2, g = x_i.x_j, the plane rotation
//   x_i <- c x_i - s x_j,  x_j <- s x_i + c x_j,
//   t = s / c the root of smaller magnitude of t^2 + 2 zeta t - 1 = 0,
//   zeta = (b - a) / (2 g),
// makes the two columns orthogonal; the same rotation applied to the
// columns of Vh (starting from the identity) accumulates X_0 Vh = X.  Sweeps
// visit every pair once in the round-robin (circle) order, all pairs of a
// round at once (one lane group each, disjoint columns); they stop after a sweep
// without a rotation (|g| <= tol sqrt(a b)).  Then sigma_j = |x_j|.  The
// arithmetic of every pair is a fixed sequence, so results repeat bit for
// bit.  A sector whose X does not fit LDS would pull every round's columns
// through one CU's L2; such sectors instead run a round per launch, each
// pair of the round on a workgroup of its own (svd_round_kernel).
#include <algorithm>
#include <cfloat>
#include <type_traits>

#include "plan.h"

#include "svd.h"

namespace bst {

namespace {
__device__ __forceinline__ double wave_allsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
}  // namespace

__global__ __launch_bounds__(256) void svd_gather_kernel(const SvdGather* __restrict__ jobs,
                                                         const SvdWork* __restrict__ work,
                                                         const double* __restrict__ in, double* __restrict__ X) {
  const SvdWork w = work[blockIdx.x];
  const SvdGather j = jobs[w.job];
  const int64_t total = (int64_t)j.rows * j.cols;
  for (int e = threadIdx.x; e < kSvdGatherChunk; e += 256) {
    const int64_t idx = (int64_t)w.start + e;
    if (idx >= total) break;
    const int64_t r = idx / j.cols, c = idx % j.cols;
    const int64_t R = j.row0 + r, C = j.col0 + c;
    const int64_t dst = j.m >= j.n ? R + C * j.m : C + R * j.n;
    X[j.x_off + dst] = in[j.in_off + idx];
  }
}

#define BST_LDS __attribute__((address_space(3)))

// The sweeps of one sector on X (p x r, column-major) and Vh (r x r): P is a
// pointer to global memory or, for sectors held in LDS, an LDS-addressed
// pointer (so that the compiler issues LDS accesses, not generic ones).
// Returns the sweeps used.
// Sum over groups of LP lanes (LP = 16, 32, 64; every lane of a group gets
// the same value).
template <int LP>
__device__ __forceinline__ double group_allsum(double v) {
#pragma unroll
  for (int off = LP / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LP);
  return v;
}

// The sweeps of one sector on X (p x r, column-major) and Vh (r x r): PX
// and PV are pointers to global memory or, for what is held in LDS,
// LDS-addressed pointers (so that the compiler issues LDS accesses, not
// generic ones).  One group of LP lanes per pair of a round.  Returns the
// sweeps used.
template <int LP, typename PX, typename PV>
__device__ int jacobi_sweeps(PX x, PV vh, int p, int r, int* rotated) {
  constexpr int NH = 64 * kSvdWaves / LP;   // lane groups of the workgroup
  const int tid = threadIdx.x, hl = tid % LP, half = tid / LP;
  const double tol = 4.0 * DBL_EPSILON * sqrt((double)p);
  const int rr = r + (r & 1);   // an odd count gets one idle slot
  int sw = 0;
  for (; sw < kSvdMaxSweeps && r > 1; ++sw) {
    for (int t = 0; t < rr - 1; ++t) {
      for (int k = half; k < rr / 2; k += NH) {
        // circle method: slot 0 stays, the others advance by one per round
        const int s0 = k, s1 = rr - 1 - k;
        int i = s0 == 0 ? 0 : (s0 - 1 + t) % (rr - 1) + 1;
        int j = (s1 - 1 + t) % (rr - 1) + 1;
        if (i > j) {
          const int q = i;
          i = j;
          j = q;
        }
        if (j >= r) continue;
        PX xi = x + (int64_t)i * p;
        PX xj = x + (int64_t)j * p;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int e = hl; e < p; e += LP) {
          const double u = xi[e], v = xj[e];
          a += u * u;
          b += v * v;
          g += u * v;
        }
        a = group_allsum<LP>(a);
        b = group_allsum<LP>(b);
        g = group_allsum<LP>(g);
        if (a == 0.0 || b == 0.0 || !(fabs(g) > tol * sqrt(a) * sqrt(b))) continue;
        const double zeta = (b - a) / (2.0 * g);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
        for (int e = hl; e < p; e += LP) {
          const double u = xi[e], v = xj[e];
          xi[e] = c * u - s * v;
          xj[e] = s * u + c * v;
        }
        PV vi = vh + (int64_t)i * r;
        PV vj = vh + (int64_t)j * r;
        for (int e = hl; e < r; e += LP) {
          const double u = vi[e], v = vj[e];
          vi[e] = c * u - s * v;
          vj[e] = s * u + c * v;
        }
        if (hl == 0) *rotated = 1;
      }
      __syncthreads();
    }
    const bool done = *rotated == 0;
    __syncthreads();
    if (tid == 0) *rotated = 0;
    __syncthreads();
    if (done) break;
  }
  return sw;
}

__global__ __launch_bounds__(64 * kSvdWaves) void svd_jacobi_kernel(const SvdSec* __restrict__ secs, double* X,
                                                                   double* V, double* __restrict__ sig,
                                                                   double* __restrict__ sorted,
                                                                   int32_t* __restrict__ perm,
                                                                   int32_t* __restrict__ sweeps, int only) {
  constexpr int NT = 64 * kSvdWaves;
  const SvdSec S = secs[blockIdx.x];
  const int p = S.m >= S.n ? S.m : S.n, r = S.m >= S.n ? S.n : S.m;
  // only = 1: the sectors that fit (their sweeps); 2: the big ones (sigma
  // and order after their rounds); 0: all
  if ((only == 1 && svd_sector_is_big(S.m, S.n)) || (only == 2 && !svd_sector_is_big(S.m, S.n))) return;
  double* const xg = X + S.x_off;
  double* const vg = V + S.v_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int rotated;
  // X is rotated in LDS when it fits kSvdLdsBytes, and Vh with it when both
  // fit; what does not fit works in global memory (the three dots of a pair
  // read X only, so X in LDS keeps them off global latency).  Copied back
  // at the end.
  __shared__ double lds[kSvdLdsBytes / sizeof(double)];
  const bool x_lds = (int64_t)p * r * (int64_t)sizeof(double) <= kSvdLdsBytes;
  const bool v_lds = x_lds && ((int64_t)p * r + (int64_t)r * r) * (int64_t)sizeof(double) <= kSvdLdsBytes;
  BST_LDS double* xl = (BST_LDS double*)lds;
  BST_LDS double* vl = xl + (int64_t)p * r;
  // a big sector arrives rotated (svd_round_kernel), its sweeps counted
  const bool pre = svd_sector_is_big(S.m, S.n);
  if (x_lds)
    for (int64_t e = tid; e < (int64_t)p * r; e += NT) xl[e] = xg[e];
  if (v_lds)
    for (int64_t e = tid; e < (int64_t)r * r; e += NT) vl[e] = (e % r == e / r) ? 1.0 : 0.0;
  else if (!pre)
    for (int64_t e = tid; e < (int64_t)r * r; e += NT) vg[e] = (e % r == e / r) ? 1.0 : 0.0;
  if (tid == 0) rotated = 0;
  __syncthreads();
  // the widest lane groups that still give every pair of a round its own
  // group (wide groups for few long columns, narrow ones for many short)
  const int npairs = (r + 1) / 2;
  auto sweeps_lp = [&](auto lp) {
    constexpr int L = decltype(lp)::value;
    if (v_lds) return jacobi_sweeps<L>(xl, vl, p, r, &rotated);
    if (x_lds) return jacobi_sweeps<L>(xl, vg, p, r, &rotated);
    return jacobi_sweeps<L>(xg, vg, p, r, &rotated);
  };
  int sw;
  if (pre)
    sw = sweeps[blockIdx.x];
  else if (npairs <= NT / 64)
    sw = sweeps_lp(std::integral_constant<int, 64>());
  else if (npairs <= NT / 32)
    sw = sweeps_lp(std::integral_constant<int, 32>());
  else
    sw = sweeps_lp(std::integral_constant<int, 16>());
  // sigma_j = |x_j| (one column per wave), from where the sweeps left X
  for (int j = wave; j < r; j += kSvdWaves) {
    double a = 0.0;
    if (x_lds) {
      for (int e = lane; e < p; e += 64) a += xl[(int64_t)j * p + e] * xl[(int64_t)j * p + e];
    } else {
      for (int e = lane; e < p; e += 64) a += xg[(int64_t)j * p + e] * xg[(int64_t)j * p + e];
    }
    a = wave_allsum(a);
    if (lane == 0) sig[S.s_off + j] = sqrt(a);
  }
  if (x_lds)
    for (int64_t e = tid; e < (int64_t)p * r; e += NT) xg[e] = xl[e];
  if (v_lds)
    for (int64_t e = tid; e < (int64_t)r * r; e += NT) vg[e] = vl[e];
  __syncthreads();
  // descending order, ties by column: rank of every value
  for (int j = tid; j < r; j += NT) {
    const double v = sig[S.s_off + j];
    int rank = 0;
    for (int i = 0; i < r; ++i) {
      const double w = sig[S.s_off + i];
      rank += (w > v || (w == v && i < j)) ? 1 : 0;
    }
    perm[S.s_off + rank] = j;
    sorted[S.s_off + rank] = v;
  }
  if (tid == 0) sweeps[blockIdx.x] = sw;
}

// Rounds of the big sectors, a launch per round.  Block (k, b) takes pair k
// of round t of big sector b (the circle order of jacobi_sweeps) with 256
// lanes: the three sums over the column (lane-strided, then the wave sums
// and the four waves in order), the same test and rotation, both columns of
// X and of Vh updated.  Any rotation sets the sector's flag for the sweep.
__global__ __launch_bounds__(256) void svd_round_kernel(const SvdSec* __restrict__ secs,
                                                        const int32_t* __restrict__ big, double* X, double* V,
                                                        int t, int32_t* flags) {
  const int b = blockIdx.y;
  if (flags[2 * b + 1]) return;   // converged
  const SvdSec S = secs[big[b]];
  const int p = S.m >= S.n ? S.m : S.n, r = S.m >= S.n ? S.n : S.m;
  const int rr = r + (r & 1);
  const int k = blockIdx.x;
  if (t >= rr - 1 || k >= rr / 2) return;
  const int s0 = k, s1 = rr - 1 - k;
  int i = s0 == 0 ? 0 : (s0 - 1 + t) % (rr - 1) + 1;
  int j = (s1 - 1 + t) % (rr - 1) + 1;
  if (i > j) {
    const int q = i;
    i = j;
    j = q;
  }
  if (j >= r) return;
  double* const xi = X + S.x_off + (int64_t)i * p;
  double* const xj = X + S.x_off + (int64_t)j * p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double a = 0.0, bb = 0.0, g = 0.0;
  for (int e = tid; e < p; e += 256) {
    const double u = xi[e], v = xj[e];
    a += u * u;
    bb += v * v;
    g += u * v;
  }
  a = wave_allsum(a);
  bb = wave_allsum(bb);
  g = wave_allsum(g);
  __shared__ double red[3][4];
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = bb;
    red[2][wave] = g;
  }
  __syncthreads();
  a = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  bb = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  g = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
  const double tol = 4.0 * DBL_EPSILON * sqrt((double)p);
  if (a == 0.0 || bb == 0.0 || !(fabs(g) > tol * sqrt(a) * sqrt(bb))) return;
  const double zeta = (bb - a) / (2.0 * g);
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
  for (int e = tid; e < p; e += 256) {
    const double u = xi[e], v = xj[e];
    xi[e] = c * u - sn * v;
    xj[e] = sn * u + c * v;
  }
  double* const vi = V + S.v_off + (int64_t)i * r;
  double* const vj = V + S.v_off + (int64_t)j * r;
  for (int e = tid; e < r; e += 256) {
    const double u = vi[e], v = vj[e];
    vi[e] = c * u - sn * v;
    vj[e] = sn * u + c * v;
  }
  if (tid == 0) flags[2 * b] = 1;
}

// Identity Vh and cleared flags and counts of the big sectors (grid y: the
// sector, x: pieces of its r x r).
__global__ __launch_bounds__(256) void svd_big_init_kernel(const SvdSec* __restrict__ secs,
                                                           const int32_t* __restrict__ big, double* V,
                                                           int32_t* flags, int32_t* sweeps) {
  const int b = blockIdx.y;
  const SvdSec S = secs[big[b]];
  const int64_t r = S.m >= S.n ? S.n : S.m;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < r * r; e += (int64_t)gridDim.x * 256)
    V[S.v_off + e] = (e % r == e / r) ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[2 * b] = 0;
    flags[2 * b + 1] = 0;
    sweeps[big[b]] = 0;
  }
}

// End of a sweep of the big sectors: a sector that rotated counts the
// sweep, one that did not is converged (as jacobi_sweeps stops).
__global__ __launch_bounds__(256) void svd_sweep_end_kernel(int nbig, const int32_t* __restrict__ big,
                                                            int32_t* flags, int32_t* sweeps) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < nbig; b += gridDim.x * 256) {
    if (!flags[2 * b + 1]) {
      if (flags[2 * b])
        sweeps[big[b]] += 1;
      else
        flags[2 * b + 1] = 1;
    }
    flags[2 * b] = 0;
  }
}

hipError_t launch_svd_gather(const SvdLaunch& l, hipStream_t s) {
  if (l.ngwork > 0x7FFFFFFF || l.nsec < 0 || l.nbig < 0 || l.nbig > 65535) return hipErrorInvalidValue;
  if (l.ngwork > 0)
    hipLaunchKernelGGL(svd_gather_kernel, dim3((unsigned)l.ngwork), dim3(256), 0, s, l.gjobs, l.gwork, l.in, l.X);
  if (l.nbig > 0) {
    const int64_t gx = std::min<int64_t>(std::max<int64_t>((l.vmax + 4095) / 4096, 1), 1024);
    hipLaunchKernelGGL(svd_big_init_kernel, dim3((unsigned)gx, (unsigned)l.nbig), dim3(256), 0, s, l.secs, l.big,
                       l.V, l.flags, l.sweeps);
  }
  return hipGetLastError();
}

hipError_t launch_svd_sweep(const SvdLaunch& l, hipStream_t s) {
  if (l.nbig <= 0) return hipSuccess;
  if (l.nbig > 65535 || l.pairs <= 0 || l.rounds <= 0) return hipErrorInvalidValue;
  for (int t = 0; t < l.rounds; ++t)
    hipLaunchKernelGGL(svd_round_kernel, dim3((unsigned)l.pairs, (unsigned)l.nbig), dim3(256), 0, s, l.secs, l.big,
                       l.X, l.V, t, l.flags);
  hipLaunchKernelGGL(svd_sweep_end_kernel, dim3((unsigned)((l.nbig + 255) / 256)), dim3(256), 0, s, l.nbig, l.big,
                     l.flags, l.sweeps);
  return hipGetLastError();
}

hipError_t launch_svd_finish(const SvdLaunch& l, hipStream_t s, int only) {
  if (l.nsec < 0 || only < 0 || only > 2) return hipErrorInvalidValue;
  if (l.nsec > 0)
    hipLaunchKernelGGL(svd_jacobi_kernel, dim3((unsigned)l.nsec), dim3(64 * kSvdWaves), 0, s, l.secs, l.X, l.V,
                       l.sig, l.sorted, l.perm, l.sweeps, only);
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// Truncation across sectors (one workgroup).  Every sector first keeps its
// min_blockdim largest values; the other values not below err are the
// candidates, ordered by value (descending), then sector, then position; the
// first keepdim - (forced) of them are kept.  The cut is found by bisection
// on the bit pattern of the values (non-negative doubles order like their
// bits), then on the flat position among values equal to the cut.
// ------------------------------------------------------------------------
constexpr int kSelectMaxSectors = 4096;
constexpr int kSelectLdsValues = 8192;   // values staged in LDS when they all fit

__global__ __launch_bounds__(1024) void svd_select_kernel(const SvdSec* __restrict__ secs, int nsec,
                                                         const double* __restrict__ sorted,
                                                         const int64_t* __restrict__ min_blockdim,
                                                         int64_t keepdim, double err, int64_t* __restrict__ kept,
                                                         double* __restrict__ s_err) {
  __shared__ unsigned long long red[16];
  __shared__ int cnt[kSelectMaxSectors];
  __shared__ long long forced_total, total;
  __shared__ double vals[kSelectLdsValues];
  // per sector: value offset (below 2^31: the plan refuses more values),
  // rank and forced count, staged once, since every counting pass of the
  // bisections below walks all sectors
  __shared__ int soff[kSelectMaxSectors], srank[kSelectMaxSectors], sforced[kSelectMaxSectors];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = tid; q < nsec; q += 1024) {
    const SvdSec S = secs[q];
    const int r = S.m < S.n ? S.m : S.n;
    const int64_t f = min_blockdim ? min_blockdim[q] : 0;
    soff[q] = (int)S.s_off;
    srank[q] = r;
    sforced[q] = (int)(f < 0 ? 0 : (f < r ? f : r));
  }
  __syncthreads();
  auto rsec = [&](int q) { return srank[q]; };
  // the sorted values of all sectors (flat, s_off + i) in LDS when they fit:
  // every bisection step below scans them all
  if (tid == 0) {
    long long t = 0;
    for (int q = 0; q < nsec; ++q) t = (long long)soff[q] + rsec(q) > t ? (long long)soff[q] + rsec(q) : t;
    total = t;
  }
  __syncthreads();
  const bool staged = total <= kSelectLdsValues;
  if (staged)
    for (long long e = tid; e < total; e += 1024) vals[e] = sorted[e];
  const double* src = staged ? (const double*)vals : sorted;
  auto forced = [&](int q) -> int { return sforced[q]; };
  // block-wide sum of per-thread counts
  auto block_sum = [&](unsigned long long v) -> unsigned long long {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < 16; ++w) t += red[w];
    return t;
  };
  // candidates with bits >= lo (mode 0), or with bits == lo and flat < lim (mode 1)
  auto count = [&](int mode, unsigned long long lo, long long lim) -> unsigned long long {
    unsigned long long c = 0;
    for (int q = 0; q < nsec; ++q) {
      const int r = rsec(q), f = forced(q);
      for (int i = f + tid; i < r; i += 1024) {
        const double v = src[(long long)soff[q] + i];
        if (!(v >= err)) continue;
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        if (mode == 0) c += b >= lo ? 1 : 0;
        else c += (b == lo && (long long)soff[q] + i < lim) ? 1 : 0;
      }
    }
    return block_sum(c);
  };
  for (int q = tid; q < nsec; q += 1024) cnt[q] = 0;
  if (tid == 0) {
    long long ft = 0;
    for (int q = 0; q < nsec; ++q) ft += forced(q);
    forced_total = ft;
  }
  __syncthreads();
  const long long room = keepdim - forced_total;
  const unsigned long long ncand = count(0, 0ull, 0);
  unsigned long long cut = 0ull;
  long long lim = 0;
  bool all = room >= (long long)ncand, none = room <= 0;
  if (!all && !none) {
    // the room-th largest candidate value: the largest bit pattern T with
    // count(>= T) >= room
    unsigned long long lo = 0ull, hi = 0x7FF0000000000000ull;
    while (lo < hi) {
      const unsigned long long mid = lo + (hi - lo + 1) / 2;
      if (count(0, mid, 0) >= (unsigned long long)room) lo = mid;
      else hi = mid - 1;
    }
    cut = lo;
    const long long need = room - (long long)count(0, cut + 1, 0);
    // the smallest flat bound with need equal values before it
    long long a = 0, b = 0;
    for (int q = 0; q < nsec; ++q) b = (long long)soff[q] + rsec(q) > b ? (long long)soff[q] + rsec(q) : b;
    while (a < b) {
      const long long mid = a + (b - a) / 2;
      if ((long long)count(1, cut, mid) >= need) b = mid;
      else a = mid + 1;
    }
    lim = a;
  }
  for (int q = 0; q < nsec; ++q) {
    const int r = rsec(q), f = forced(q);
    int c = 0;
    for (int i = f + tid; i < r; i += 1024) {
      const double v = src[(long long)soff[q] + i];
      if (!(v >= err) || none) continue;
      const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
      c += (all || bits > cut || (bits == cut && (long long)soff[q] + i < lim)) ? 1 : 0;
    }
    if (c) atomicAdd(&cnt[q], c);
  }
  __syncthreads();
  if (tid == 0) {
    double e = 0.0;
    for (int q = 0; q < nsec; ++q) {
      const int k = forced(q) + cnt[q];
      kept[q] = k;
      if (k < rsec(q)) e = fmax(e, sorted[(long long)soff[q] + k]);
    }
    *s_err = e;
  }
}

hipError_t launch_svd_select(const SvdSelectLaunch& l, hipStream_t s) {
  if (l.nsec < 0 || l.nsec > kSelectMaxSectors) return hipErrorInvalidValue;
  hipLaunchKernelGGL(svd_select_kernel, dim3(1), dim3(1024), 0, s, l.secs, l.nsec, l.sorted, l.min_blockdim,
                     l.keepdim, l.err, l.kept, l.s_err);
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// Kept columns into the output factors
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void svd_write_kernel(const SvdWrite* __restrict__ jobs,
                                                        const SvdWriteWork* __restrict__ work,
                                                        const SvdSec* __restrict__ secs, const double* __restrict__ X,
                                                        const double* __restrict__ V,
                                                        const double* __restrict__ sorted,
                                                        const int32_t* __restrict__ perm, int absorb, double* U,
                                                        double* Vd, double* Sv) {
  const SvdWriteWork w = work[blockIdx.x];
  const SvdWrite j = jobs[w.job];
  const SvdSec S = secs[j.sec];
  const bool tall = S.m >= S.n;
  const int64_t p = tall ? S.m : S.n, r = tall ? S.n : S.m;
  const int64_t total = j.kind == 2 ? j.k : (int64_t)j.ext * j.k;
  for (int e = threadIdx.x; e < kSvdGatherChunk; e += 256) {
    const int64_t idx = (int64_t)w.start + e;
    if (idx >= total) break;
    if (j.kind == 2) {
      Sv[j.out_off + idx] = sorted[S.s_off + idx];
      continue;
    }
    // U: (row, c) = (idx / k, idx % k); V^dagger: (c, col) = (idx / ext, idx % ext)
    const int64_t c = j.kind == 0 ? idx % j.k : idx / j.ext;
    const int64_t row = j.off0 + (j.kind == 0 ? idx / j.k : idx % j.ext);
    const int64_t col = perm[S.s_off + c];
    const double sg = sorted[S.s_off + c];
    // U = x_j / sigma_j (tall) or Vh (wide); V = Vh (tall) or x_j / sigma_j (wide)
    const bool from_x = (j.kind == 0) == tall;
    double v;
    if (from_x) {
      v = sg > 0.0 ? X[S.x_off + row + col * p] / sg : 0.0;
    } else {
      v = V[S.v_off + row + col * r];
    }
    if ((j.kind == 0 && absorb == 1) || (j.kind == 1 && absorb == 2)) v *= sg;
    (j.kind == 0 ? U : Vd)[j.out_off + idx] = v;
  }
}

hipError_t launch_svd_write(const SvdWriteLaunch& l, hipStream_t s) {
  if (l.nwork <= 0) return hipSuccess;
  if (l.nwork > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(svd_write_kernel, dim3((unsigned)l.nwork), dim3(256), 0, s, l.jobs, l.work, l.secs, l.X, l.V,
                     l.sorted, l.perm, l.absorb, l.U, l.Vd, l.S);
  return hipGetLastError();
}

}  // namespace bst

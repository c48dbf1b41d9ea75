// Symmetric SVD (Sec. "Singular value decomposition"): device records shared
// by the host plan (svd.cpp) and the kernels (kernels_svd.hip).
//
// A tensor seen as a matrix (first rowrank legs = rows) splits into one block
// matrix M_q per charge q of the new bond.  Each M_q (m x n) is held in the
// workspace as X, the "tall" orientation (p x r, p = max(m, n), r = min(m, n),
// column-major): X = M_q when m >= n, X = M_q^T otherwise.  One-sided Jacobi
// rotates the columns of X until they are orthogonal and accumulates the
// rotations in Vh (r x r, column-major); then sigma_j = |x_j|, and
//   tall: U = x_j / sigma_j, V = Vh;      wide: U = Vh, V = x_j / sigma_j.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bst {

// One block of the input, copied into its sector's X.
struct SvdGather {
  int64_t in_off;   // element offset of the block in the input tensor
  int64_t x_off;    // element offset of the sector's X in the workspace
  int32_t rows, cols;   // the block as a matrix: row-leg extent x column-leg extent
  int32_t row0, col0;   // its place in M_q
  int32_t m, n;         // M_q's shape
};
struct SvdWork {
  int32_t job, start;   // 256 * 16 elements of one job per workgroup
};

// One sector matrix.
struct SvdSec {
  int64_t x_off;    // X (p x r) in the X region
  int64_t v_off;    // Vh (r x r) in the V region
  int64_t s_off;    // r values in the sigma / sorted / perm regions
  int32_t m, n;
};

// One block of an output factor, written from its sector's X and Vh.
// kind 0: U block [row tuple..., k] (row-major as [ext x k]) from rows
// off0 .. off0 + ext of U_q; kind 1: V^dagger block [k, column tuple...]
// (row-major as [k x ext]) from rows off0 .. of V_q; kind 2: the k largest
// values of the sector into S (ext = k).
struct SvdWrite {
  int64_t out_off;
  int32_t sec, kind;
  int32_t off0, ext;
  int32_t k, pad;
};
struct SvdWriteWork {
  int32_t job, start;
};

constexpr int kSvdWaves = 16;             // waves of the Jacobi workgroup
constexpr int kSvdLdsBytes = 128 * 1024;  // X and Vh of a sector up to this size are rotated in LDS
constexpr int kSvdMaxSweeps = 60;
constexpr int kSvdGatherChunk = 256 * 16;

struct SvdLaunch {
  const SvdGather* gjobs;
  const SvdWork* gwork;
  int64_t ngwork;
  const SvdSec* secs;
  int32_t nsec;
  const double* in;
  double* X;
  double* V;
  double* sig;        // |x_j| per column
  double* sorted;     // the same values in descending order
  int32_t* perm;      // column of X (or Vh) of the c-th largest value
  int32_t* sweeps;    // per sector: sweeps used (diagnostic)
  // sectors whose X exceeds kSvdLdsBytes (and r > 1): rotated a round per
  // launch by the whole device before the per-sector kernel
  const int32_t* big;   // their sector indices
  int32_t nbig;
  int32_t rounds;       // most rounds per sweep over them (r + (r & 1) - 1)
  int32_t pairs;        // most pairs per round
  int64_t vmax;         // largest r * r
  int32_t* flags;       // per big sector: [rotated this sweep, converged]
};
// The gather, and the identity Vh and cleared flags of the big sectors.
hipError_t launch_svd_gather(const SvdLaunch& l, hipStream_t s);
// One sweep over the big sectors not yet converged: every round, then the
// sweep's count (a sector whose sweep rotated nothing is marked converged).
hipError_t launch_svd_sweep(const SvdLaunch& l, hipStream_t s);
// The sweeps of the other sectors (one workgroup each), then sigma and the
// sorted order of every sector; only = 1 restricts it to the sectors that
// are not big, 2 to the big ones (after their rounds), 0 takes all.
hipError_t launch_svd_finish(const SvdLaunch& l, hipStream_t s, int only);

// True when sector (m, n)'s sweeps run a round per launch on the device
// rather than in one workgroup (its X does not fit kSvdLdsBytes).
__host__ __device__ inline bool svd_sector_is_big(int64_t m, int64_t n) {
  const int64_t p = m >= n ? m : n, r = m >= n ? n : m;
  return r > 1 && p * r * 8 > kSvdLdsBytes;
}

struct SvdSelectLaunch {
  const SvdSec* secs;
  int32_t nsec;
  const double* sorted;        // per sector, descending
  const int64_t* min_blockdim; // nsec entries (device)
  int64_t keepdim;
  double err;
  int64_t* kept;               // nsec entries
  double* s_err;
};
hipError_t launch_svd_select(const SvdSelectLaunch& l, hipStream_t s);

struct SvdWriteLaunch {
  const SvdWrite* jobs;
  const SvdWriteWork* work;
  int64_t nwork;
  const SvdSec* secs;
  const double* X;
  const double* V;
  const double* sorted;
  const int32_t* perm;
  int32_t absorb;   // 0 none, 1 into U, 2 into V^dagger
  double* U;
  double* Vd;
  double* S;
};
hipError_t launch_svd_write(const SvdWriteLaunch& l, hipStream_t s);

}  // namespace bst

// Lanczos ground state of a two-site H_eff (Sec. "Eigenvalue decomposition":
// the lowest eigenpair of a Hermitian linear operator given as a matvec).
//
// The matvec runs in the requested arithmetic form; the reorthogonalisation
// against all Krylov vectors, the scalars, the tridiagonal eigensolve (on
// the host), the Ritz vector and the Rayleigh-quotient refinement with one
// float64 apply run in float64.  The Krylov rows are float64; on request,
// with the split matvec forms, they are stored in float32 instead (rounding
// them adds 6e-8 per element, far below the matvec's own 2^-17 error; every
// dot product and scalar stays float64).  All vectors stay in the
// caller's workspace; alpha/beta stay on the device until the end, so a
// step costs no host round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "plan.h"

namespace bst {

namespace {

struct LanczosLayout {
  size_t tables, V, W, Y, HY, scal, cmat, partial, dpart, end;
  int64_t ldv;   // row stride of V: psi's size rounded up to 512 bytes
  int nslots;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

LanczosLayout layout(const PlanData& P, int nsteps) {
  LanczosLayout L{};
  const size_t n = (size_t)P.psi_numel;
  L.ldv = (int64_t)((n + 63) / 64 * 64);
  size_t off = al(P.ws_bytes);
  L.nslots = std::max(P.nslots, 1);
  L.tables = off;
  off = al(off + sizeof(void*) * (size_t)L.nslots * (size_t)(nsteps + 1));
  L.V = off;
  off = al(off + sizeof(double) * (size_t)L.ldv * (size_t)nsteps);
  L.W = off;
  off = al(off + sizeof(double) * std::max<size_t>(n, 1));
  L.Y = off;
  off = al(off + sizeof(double) * std::max<size_t>(n, 1));
  L.HY = off;
  off = al(off + sizeof(double) * std::max<size_t>(n, 1));
  L.scal = off;
  // c, d, alpha, beta, s [kMaxVecs each], misc[16], cproj[kMaxVecs],
  // dn[kMaxVecs + 2]
  off = al(off + sizeof(double) * (7 * (size_t)kMaxVecs + 32));
  L.cmat = off;   // the one-pass schedule's row-to-basis map, kMaxVecs x kMaxVecs
  off = al(off + sizeof(double) * (size_t)kMaxVecs * kMaxVecs);
  L.partial = off;
  off = al(off + sizeof(double) * (size_t)(kMaxVecs + 1) * kVecBlocks);
  L.dpart = off;   // partials of the u_j.z dot
  off = al(off + sizeof(double) * 2 * (size_t)kVecBlocks);
  L.end = off;
  return L;
}

// Number of eigenvalues of the tridiagonal (a, b) below x: negative pivots
// of the LDL^T factorisation of T - x I (Sturm sequence).
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int neg = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off2 = i ? b[i - 1] * b[i - 1] : 0.0;
    q = (a[i] - x) - (i ? off2 / q : 0.0);
    if (q == 0.0) q = -std::numeric_limits<double>::min();
    if (q < 0.0) ++neg;
  }
  return neg;
}

// Lowest eigenpair: bisection on the Sturm count to the last bit, then
// inverse iteration with a pivoted tridiagonal solve.
void lowest_eigenpair(const std::vector<double>& a, const std::vector<double>& b, double& theta,
                      std::vector<double>& v) {
  const size_t n = a.size();
  v.assign(n, 1.0);
  if (n == 1) {
    theta = a[0];
    return;
  }
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < n; ++i) {
    double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 4000; ++it) {
    const double mid = lo + 0.5 * (hi - lo);
    if (!(mid > lo && mid < hi)) break;
    if (sturm_below(a, b, mid) >= 1) hi = mid;
    else lo = mid;
  }
  theta = hi;
  const double shift = theta - 4.0 * std::numeric_limits<double>::epsilon() * std::max(1.0, std::fabs(theta));
  // (T - shift) x = v by Gaussian elimination with partial pivoting on the
  // band: dl sub-diagonal, d diagonal, du super-diagonal, du2 the second
  // super-diagonal that row swaps create.
  for (int iter = 0; iter < 3; ++iter) {
    std::vector<double> dl(n, 0.0), d(n), du(n, 0.0), du2(n, 0.0), x = v;
    for (size_t i = 0; i < n; ++i) {
      d[i] = a[i] - shift;
      if (i + 1 < n) du[i] = dl[i] = b[i];
    }
    for (size_t i = 0; i + 1 < n; ++i) {
      if (std::fabs(d[i]) >= std::fabs(dl[i])) {
        if (d[i] == 0.0) d[i] = std::numeric_limits<double>::min();
        const double f = dl[i] / d[i];
        d[i + 1] -= f * du[i];
        x[i + 1] -= f * x[i];
      } else {
        // rows i and i+1 change places
        const double f = d[i] / dl[i];
        d[i] = dl[i];
        const double t = d[i + 1];
        d[i + 1] = du[i] - f * t;
        if (i + 2 < n) {
          du2[i] = du[i + 1];
          du[i + 1] = -f * du2[i];
        }
        du[i] = t;
        const double xi = x[i];
        x[i] = x[i + 1];
        x[i + 1] = xi - f * x[i + 1];
      }
    }
    if (d[n - 1] == 0.0) d[n - 1] = std::numeric_limits<double>::min();
    x[n - 1] /= d[n - 1];
    x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / d[n - 2];
    for (size_t k = n - 2; k-- > 0;) x[k] = (x[k] - du[k] * x[k + 1] - du2[k] * x[k + 2]) / d[k];
    double nrm = 0.0;
    for (double e : x) nrm += e * e;
    nrm = std::sqrt(nrm);
    for (size_t i = 0; i < n; ++i) v[i] = x[i] / nrm;
  }
  size_t imax = 0;
  for (size_t i = 1; i < n; ++i)
    if (std::fabs(v[i]) > std::fabs(v[imax])) imax = i;
  if (v[imax] < 0)
    for (auto& e : v) e = -e;
}

// HIP-event timing of kernel classes (enabled by BST_LANCZOS_TIMING).
struct ClassTimer {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<int> cls;
  size_t used = 0;
  void reserve(size_t n) {
    pool.resize(n);
    for (auto& e : pool) {
      check_hip(hipEventCreate(&e.first), "event");
      check_hip(hipEventCreate(&e.second), "event");
    }
    cls.assign(n, -1);
  }
  ~ClassTimer() {
    for (auto& e : pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
  std::pair<hipEvent_t, hipEvent_t>* take(int c) {
    if (!on || used >= pool.size()) return nullptr;
    cls[used] = c;
    return &pool[used++];
  }
  void begin(std::pair<hipEvent_t, hipEvent_t>* e, hipStream_t s) {
    if (e) check_hip(hipEventRecord(e->first, s), "event");
  }
  void end(std::pair<hipEvent_t, hipEvent_t>* e, hipStream_t s) {
    if (e) check_hip(hipEventRecord(e->second, s), "event");
  }
  void collect(double* ms, int32_t* calls) {
    for (size_t i = 0; i < used; ++i) {
      float t = 0;
      check_hip(hipEventElapsedTime(&t, pool[i].first, pool[i].second), "event time");
      ms[cls[i]] += t;
      calls[cls[i]] += 1;
    }
  }
};

int step_class(const std::string& name) {
  if (name == "gemm_L_psi") return 0;
  if (name == "mpo_apply") return 1;
  if (name == "gemm_T3_R") return 2;
  if (name == "mpo_coef" || name.compare(0, 6, "split_") == 0) return 3;
  return 7;
}

}  // namespace
}  // namespace bst

using namespace bst;

extern "C" {

bst_status bst_lanczos_workspace(const bst_plan* heff, int32_t nsteps, size_t* bytes) {
  BST_TRY
  if (!heff || !bytes) fail(BST_E_INVALID, "null argument");
  if (heff->p.kind != 2) fail(BST_E_INVALID, "Lanczos needs a single H_eff plan");
  if (nsteps < 1 || nsteps > kMaxVecs) fail(BST_E_INVALID, "nsteps must be 1..128");
  *bytes = layout(heff->p, nsteps).end;
  BST_CATCH
}

bst_status bst_lanczos_ground(bst_plan* heff, const void* const* ops, const void* psi0,
                              int32_t nsteps, bst_precision matvec_prec, int32_t refine,
                              void* psi_out, double* energy, bst_lanczos_info* info, void* ws,
                              void* stream) {
  BST_TRY
  if (!heff || !ops || !psi0 || !psi_out || !energy || !ws) fail(BST_E_INVALID, "null argument");
  PlanData& P = heff->p;
  if (P.kind != 2) fail(BST_E_INVALID, "Lanczos needs a single H_eff plan");
  if (nsteps < 1 || nsteps > kMaxVecs) fail(BST_E_INVALID, "nsteps must be 1..128");
  if (matvec_prec < BST_FP64 || matvec_prec > BST_BF16X6) fail(BST_E_INVALID, "unknown precision");
  for (int i = 0; i < 4; ++i)
    if (!ops[i]) fail(BST_E_INVALID, "null operator pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LanczosLayout Lo = layout(P, nsteps);
  char* wb = static_cast<char*>(ws);
  const int64_t n = P.psi_numel;
  const int64_t ldv = Lo.ldv;
  if ((uint64_t)ldv * (uint64_t)nsteps * 8u >= 0xFFFFFFFFull)
    fail(BST_E_INVALID, "Krylov basis above 4 GiB (reduce nsteps)");
  const bool three_pass = info && (info->flags & BST_LANCZOS_THREE_PASS);
  // Krylov rows: float64, or float32 on request with the split forms and
  // the one-pass schedule
  const bool f32_basis = info && (info->flags & BST_LANCZOS_F32_BASIS);
  const bool vf32 = !three_pass && f32_basis && (matvec_prec == BST_BF16X3 || matvec_prec == BST_BF16X6);
  double* V = reinterpret_cast<double*>(wb + Lo.V);
  float* V32 = reinterpret_cast<float*>(wb + Lo.V);
  auto row = [&](int j) -> void* {
    return vf32 ? static_cast<void*>(V32 + (size_t)j * ldv) : static_cast<void*>(V + (size_t)j * ldv);
  };
  double* W = reinterpret_cast<double*>(wb + Lo.W);
  float* W32 = reinterpret_cast<float*>(wb + Lo.W);   // H u_j with a float32 basis
  double* Y = reinterpret_cast<double*>(wb + Lo.Y);
  double* HY = reinterpret_cast<double*>(wb + Lo.HY);
  double* sc = reinterpret_cast<double*>(wb + Lo.scal);
  double* c = sc;
  double* d = sc + kMaxVecs;
  double* alpha = sc + 2 * kMaxVecs;
  double* beta = sc + 3 * kMaxVecs;
  double* svec = sc + 4 * kMaxVecs;
  double* misc = sc + 5 * kMaxVecs;   // [0..1] psi0 dot2, [2] norm2, [4..5] num, [6] r2,
                                      // [8..9] u_j.z, z.z, [10] alpha estimate
  double* cproj = misc + 16;
  double* dn = cproj + kMaxVecs;
  double* cmat = reinterpret_cast<double*>(wb + Lo.cmat);
  double* partial = reinterpret_cast<double*>(wb + Lo.partial);
  double* dpart = reinterpret_cast<double*>(wb + Lo.dpart);

  // plan tables, and one pointer table per Krylov vector plus the refinement
  const void* in0[5] = {ops[0], ops[1], ops[2], ops[3], V};
  void* out0[1] = {W};
  prepare_ws(P, in0, out0, ws, s);
  // the nsteps + 1 tables sit back to back: one upload writes them all
  std::vector<void* const*> tables;
  std::vector<void*> all;
  all.reserve((size_t)Lo.nslots * (size_t)(nsteps + 1));
  for (int j = 0; j <= nsteps; ++j) {
    const void* in[5] = {ops[0], ops[1], ops[2], ops[3], j < nsteps ? (const void*)row(j) : (const void*)Y};
    void* out[1] = {j < nsteps ? (void*)W : (void*)HY};
    auto ptrs = build_ptrs(P, in, out, ws);
    ptrs.resize((size_t)Lo.nslots, nullptr);
    all.insert(all.end(), ptrs.begin(), ptrs.end());
  }
  void* const* tab0 = static_cast<void* const*>(upload_table(P, all, ws, Lo.tables, s));
  for (int j = 0; j <= nsteps; ++j) tables.push_back(tab0 + (size_t)Lo.nslots * (size_t)j);
  ClassTimer tm;
  tm.on = info && (info->flags & BST_LANCZOS_TIMING);
  const size_t nps = P.steps.size();
  if (tm.on) tm.reserve((size_t)(nsteps + 1) * nps + (size_t)nsteps * 5 + 16);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> stepev(nps);
  auto matvec = [&](void* const* table, bst_precision prec, bool skip_coef) {
    if (!tm.on) {
      run_steps(P, ws, table, prec, s, skip_coef);
      return;
    }
    for (size_t k = 0; k < nps; ++k) {
      const bool skipped = !step_runs(P, P.steps[k], prec, skip_coef);
      auto* e = skipped ? nullptr : tm.take(step_class(P.steps[k].name));
      // unused pairs still get recorded by run_steps; give them a spare
      stepev[k] = e ? *e : tm.pool.back();
    }
    run_steps(P, ws, table, prec, s, skip_coef, &stepev);
  };
  auto timed = [&](int cls, auto&& launch) {
    auto* e = tm.take(cls);
    tm.begin(e, s);
    launch();
    tm.end(e, s);
  };
  // v1 = psi0 / |psi0|
  timed(7, [&] {
    check_hip(launch_dot2(static_cast<const double*>(psi0), static_cast<const double*>(psi0), n,
                          partial, misc, s),
              "norm");
    if (vf32)
      check_hip(launch_scale_rnorm(static_cast<const double*>(psi0), misc + 1, V32, n, s), "scale");
    else
      check_hip(launch_scale_rnorm(static_cast<const double*>(psi0), misc + 1, V, n, s), "scale");
  });
  // with a float32 basis the matvec reads float32 rows and writes H u_j as
  // float32 while the solve runs.  With float64 rows and a split form, H u_j
  // is still written as float32: the split GEMMs accumulate in float32, so
  // the stored values are the same (BST_LANCZOS_Z64 keeps it float64).
  const bool z32 = !three_pass && !vf32 && (matvec_prec == BST_BF16X3 || matvec_prec == BST_BF16X6) &&
                   !std::getenv("BST_LANCZOS_Z64");
  struct Psi32 {
    PlanData& P;
    Psi32(PlanData& p, bool rows32, bool z) : P(p) {
      P.psi_f32 = rows32;
      P.z_f32 = rows32 || z;
    }
    ~Psi32() { P.psi_f32 = P.z_f32 = false; }
  } psi32(P, vf32, z32);
  for (int j = 0; j < nsteps; ++j) {
    matvec(tables[j], matvec_prec, j > 0);
    const int nv = j + 1;
    double* vnext = j + 1 < nsteps ? V + (size_t)(j + 1) * ldv : nullptr;
    if (three_pass) {
      // w -= V (V^T w) twice, then alpha, beta and v_{j+1} = w / beta
      timed(4, [&] { check_hip(launch_multidot(V, ldv, n, nv, W, partial, c, s), "cgs pass 1"); });
      timed(5, [&] { check_hip(launch_project(V, ldv, n, nv, c, W, W, 1, partial, d, s), "cgs pass 2"); });
      timed(6, [&] { check_hip(launch_project(V, ldv, n, nv, d, W, W, 2, partial, nullptr, s), "cgs pass 3"); });
      timed(7, [&] {
        check_hip(launch_lanczos_step_end(partial, n, c, d, j, alpha, beta, misc + 2, W, vnext, n, s),
                  "step end");
      });
    } else {
      // row j holds u_j, W = H u_j: one launch for the dot u_j.z, the end
      // of step j - 1, row j of C and the scalars of step j, then one pass
      // over rows 0..j that forms the residual and measures it
      timed(4, [&] {
        if (vf32)
          check_hip(launch_lanczos_dot_step(V32 + (size_t)j * ldv, W32, n, dpart, partial, j - 1, dn, j,
                                            misc + 8, alpha, beta, d, cproj, misc + 10, cmat, s),
                    "step scalars");
        else if (z32)
          check_hip(launch_lanczos_dot_step(V + (size_t)j * ldv, W32, n, dpart, partial, j - 1, dn, j,
                                            misc + 8, alpha, beta, d, cproj, misc + 10, cmat, s),
                    "step scalars");
        else
          check_hip(launch_lanczos_dot_step(V + (size_t)j * ldv, W, n, dpart, partial, j - 1, dn, j,
                                            misc + 8, alpha, beta, d, cproj, misc + 10, cmat, s),
                    "step scalars");
      });
      timed(5, [&] {
        if (vf32)
          check_hip(launch_lanczos_pass(V32, ldv, n, j, W32, cproj, beta,
                                        j + 1 < nsteps ? V32 + (size_t)(j + 1) * ldv : nullptr, partial,
                                        nullptr, s),
                    "basis pass");
        else if (z32)
          check_hip(launch_lanczos_pass(V, ldv, n, j, W32, cproj, beta, vnext, partial, nullptr, s),
                    "basis pass");
        else
          check_hip(launch_lanczos_pass(V, ldv, n, j, W, cproj, beta, vnext, partial, nullptr, s),
                    "basis pass");
      });
    }
  }
  if (!three_pass) {
    // the end of the last step
    timed(7, [&] {
      check_hip(launch_lanczos_pass_sums(n, nsteps - 1, vf32, partial, dn, s), "step sums");
      check_hip(launch_lanczos_end(dn, misc + 10, nsteps - 1, cmat, d, alpha, beta, s), "step end");
    });
  }
  std::vector<double> ha(nsteps), hb(nsteps), m0(2);
  check_hip(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * nsteps, hipMemcpyDeviceToHost, s), "d2h");
  check_hip(hipMemcpyAsync(hb.data(), beta, sizeof(double) * nsteps, hipMemcpyDeviceToHost, s), "d2h");
  check_hip(hipMemcpyAsync(m0.data(), misc, sizeof(double) * 2, hipMemcpyDeviceToHost, s), "d2h");
  check_hip(hipStreamSynchronize(s), "lanczos sync");
  if (!(m0[1] > 0.0) || !std::isfinite(m0[1])) fail(BST_E_NOTCONV, "start vector is zero or not finite");
  // steps kept: up to the first breakdown
  int m = nsteps;
  double amax = 0.0;
  for (int j = 0; j < nsteps; ++j) {
    if (!std::isfinite(ha[j]) || !std::isfinite(hb[j])) fail(BST_E_NOTCONV, "non-finite Lanczos coefficient");
    amax = std::max(amax, std::fabs(ha[j]));
    if (hb[j] <= 1e-12 * std::max(amax, hb[j])) {
      m = j + 1;
      break;
    }
  }
  std::vector<double> a(ha.begin(), ha.begin() + m), b(hb.begin(), hb.begin() + (m - 1));
  double theta;
  std::vector<double> sv;
  lowest_eigenpair(a, b, theta, sv);
  // y = V s: with the one-pass schedule the rows are the residuals as
  // written and v_k = sum_{i<=k} C[k][i] u_i, so the combination takes
  // s'_i = sum_{k>=i} s_k C[k][i] over rows 0..m-1
  std::vector<double> ycoef = sv;
  if (!three_pass) {
    std::vector<double> C((size_t)m * kMaxVecs);
    check_hip(hipMemcpyAsync(C.data(), cmat, sizeof(double) * C.size(), hipMemcpyDeviceToHost, s), "d2h");
    check_hip(hipStreamSynchronize(s), "d2h sync");
    for (int i = 0; i < m; ++i) {
      double t = 0.0;
      for (int k = i; k < m; ++k) t += sv[k] * C[(size_t)k * kMaxVecs + i];
      ycoef[i] = t;
    }
  }
  check_hip(hipMemcpyAsync(svec, ycoef.data(), sizeof(double) * m, hipMemcpyHostToDevice, s), "h2d");
  check_hip(hipStreamSynchronize(s), "h2d sync");
  psi32.P.psi_f32 = psi32.P.z_f32 = false;   // the refinement: float64 in and out
  timed(7, [&] {
    if (vf32)
      check_hip(launch_combine(V32, ldv, n, m, svec, Y, s), "ritz vector");
    else
      check_hip(launch_combine(V, ldv, n, m, svec, Y, s), "ritz vector");
  });
  double E = theta, resid = -1.0;
  if (refine) {
    matvec(tables[nsteps], BST_FP64, false);
    check_hip(launch_dot2(HY, Y, n, partial, misc + 4, s), "rayleigh");
    check_hip(launch_resid(HY, Y, misc + 4, n, partial, misc + 6, s), "residual");
    double h[3];
    check_hip(hipMemcpyAsync(h, misc + 4, sizeof(double) * 3, hipMemcpyDeviceToHost, s), "d2h");
    check_hip(hipStreamSynchronize(s), "refine sync");
    E = h[0] / h[1];
    resid = std::sqrt(h[2] / h[1]);
  } else {
    check_hip(launch_dot2(Y, Y, n, partial, misc + 4, s), "norm");
    resid = hb[m - 1] * std::fabs(sv[m - 1]);
  }
  check_hip(launch_scale_rnorm(Y, misc + 5, static_cast<double*>(psi_out), n, s), "normalise");
  check_hip(hipStreamSynchronize(s), "final sync");
  *energy = E;
  if (info) {
    const int32_t flags = info->flags;
    std::memset(info, 0, sizeof(*info));
    info->flags = (flags & ~BST_LANCZOS_Z32) | (z32 ? BST_LANCZOS_Z32 : 0);
    if (tm.on) tm.collect(info->kernel_ms, info->kernel_calls);
    info->steps = m;
    info->theta = theta;
    double bmin = m > 1 ? hb[0] : hb[m - 1];
    for (int j = 0; j + 1 < m; ++j) bmin = std::min(bmin, hb[j]);
    info->beta_min = bmin;
    info->residual = resid;
    for (int j = 0; j < m && j < 128; ++j) info->alpha[j] = ha[j];
    for (int j = 0; j < m && j < 128; ++j) info->beta[j] = hb[j];
  }
  BST_CATCH
}

}  // extern "C"

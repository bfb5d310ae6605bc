// host_check.cpp -- drives the C ABI of the library through its host paths
// (validation, layout, planning of windows and tiles, graph capture, the
// tuners, the adjoint's segment bookkeeping, the allocation-free entry
// point) on small batches, so that a build of the library's host code with
// AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged)
// checks its memory accesses and arithmetic.  Test infrastructure: built by
// paper_2510_07539_amd/build.py (build_host_check) and run by
// tests/test_gpu_sanitize.py.  Prints one line per call; exits non-zero if
// a call returns an unexpected code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hsgn.h"

namespace {

int failures = 0;

void expect(const char* what, int rc, int want, hsgn_ctx* c = nullptr) {
  std::printf("%-40s rc=%d\n", what, rc);
  std::fflush(stdout);
  if (rc != want) {
    std::fprintf(stderr, "%s: rc %d, expected %d (%s)\n", what, rc, want,
                 c ? hsgn_last_error(c) : "");
    ++failures;
  }
}

struct Batch {
  std::vector<int64_t> off;
  std::vector<hsgn_params> prm;
  std::vector<double> b, h, q;
};

hsgn_params params(int bc, int bed, int order, int scheme, double lam, double dx) {
  hsgn_params p;
  p.g = 9.81;
  p.lambda = lam;
  p.dx = dx;
  p.cfl = scheme == HSGN_SCHEME_EXPLICIT ? 0.4 : 0.9;
  p.mcfl = 0.5;
  p.dt_fixed = 0.0;
  p.t_end = 0.0;
  p.bc = bc;
  p.has_bathymetry = bed;
  p.order = order;
  p.scheme = scheme;
  return p;
}

// uneven instances: a hump on 0.4 m of water, bar-like bed where asked
Batch batch(const std::vector<int>& sizes, int order, int scheme, bool bed) {
  Batch B;
  B.off.push_back(0);
  for (size_t j = 0; j < sizes.size(); ++j) {
    const int n = sizes[j];
    const int bc = (int)(j % 2);
    const bool bj = bed && bc == 1;
    const double dx = 0.04, L = n * dx;
    B.prm.push_back(params(bc, bj ? 1 : 0, order, scheme, j % 3 == 0 ? 100.0 : 1000.0, dx));
    for (int i = 0; i < n; ++i) {
      const double x = (i + 0.5) * dx;
      const double bb = bj ? 0.15 * std::exp(-std::pow((x - 0.6 * L) / (0.1 * L), 2)) : 0.0;
      const double z = 0.4 + 0.04 * std::exp(-std::pow((x - 0.3 * L) / (0.05 * L), 2));
      B.b.push_back(bb);
      B.h.push_back(z - bb);
      B.q.push_back(0.0);
    }
    B.off.push_back(B.off.back() + n);
  }
  return B;
}

void hip_or_die(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    std::exit(2);
  }
}

double* dev(const std::vector<double>& v) {
  double* d = nullptr;
  hip_or_die(hipMalloc(&d, (v.empty() ? 1 : v.size()) * sizeof(double)), "hipMalloc");
  if (!v.empty())
    hip_or_die(hipMemcpy(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice),
               "hipMemcpy");
  return d;
}

void run_context(const char* name, const Batch& B, bool tune) {
  std::printf("== %s: %zu instances, %lld cells\n", name, B.prm.size(), (long long)B.off.back());
  const int ni = (int)B.prm.size();
  double *db = dev(B.b), *dh = dev(B.h), *dq = dev(B.q);
  hsgn_ctx* c = nullptr;
  const bool any_b = [&] {
    for (auto& p : B.prm)
      if (p.has_bathymetry) return true;
    return false;
  }();
  expect("hsgn_init", hsgn_init(&c, ni, B.off.data(), B.prm.data(), any_b ? db : nullptr, nullptr),
         HSGN_OK);
  if (!c) return;
  expect("hsgn_set_state (default m, W)", hsgn_set_state(c, dh, dq, nullptr, nullptr, nullptr),
         HSGN_OK, c);
  std::vector<int32_t> mode(ni), halo(ni), flags(ni);
  int32_t counts[4];
  expect("hsgn_plan_info", hsgn_plan_info(c, mode.data(), halo.data(), counts), HSGN_OK, c);
  const int scheme = B.prm[0].scheme;
  const int32_t modes[3] = {HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT, HSGN_SOLVER_AUTO_SMALL};
  for (int32_t m : modes) {
    expect("hsgn_set_solver", hsgn_set_solver(c, m), HSGN_OK, c);
    expect("hsgn_step", hsgn_step(c, 2), HSGN_OK, c);
  }
  expect("hsgn_run (graph, twice)", hsgn_run(c, 8, 4), HSGN_OK, c);
  expect("hsgn_run (again)", hsgn_run(c, 5, 4), HSGN_OK, c);
  double ms[HSGN_NKERNEL];
  int32_t cnt[HSGN_NKERNEL];
  expect("hsgn_step_timed", hsgn_step_timed(c, 2, ms, cnt), HSGN_OK, c);
  expect("hsgn_status", hsgn_status(c, flags.data()), HSGN_OK, c);
  std::vector<double> zero(B.off.back(), 0.0);
  double *gh = dev(zero), *gq = dev(zero), *gm = dev(zero), *gW = dev(zero), *gt = dev(zero),
         *gdt = dev(zero);
  expect("hsgn_get_state", hsgn_get_state(c, gh, gq, gm, gW, gt), HSGN_OK, c);
  expect("hsgn_get_dt", hsgn_get_dt(c, gdt), HSGN_OK, c);
  expect("hsgn_set_state (all fields)", hsgn_set_state(c, gh, gq, gm, gW, gt), HSGN_OK, c);
  if (scheme == HSGN_SCHEME_SEMI_IMPLICIT) {
    std::vector<int32_t> per(ni);
    for (int j = 0; j < ni; ++j) per[j] = modes[j % 3];
    expect("hsgn_set_instance_solvers", hsgn_set_instance_solvers(c, per.data()), HSGN_OK, c);
    expect("hsgn_step (per-instance modes)", hsgn_step(c, 2), HSGN_OK, c);
    expect("hsgn_set_launch (persistent)", hsgn_set_launch(c, HSGN_LAUNCH_PERSISTENT), HSGN_OK, c);
    expect("hsgn_run (persistent)", hsgn_run(c, 4, 2), HSGN_OK, c);
    expect("hsgn_set_launch (grid)", hsgn_set_launch(c, HSGN_LAUNCH_GRID), HSGN_OK, c);
    if (tune) {
      double tms[3], lms[2], whole[5];
      int32_t kept = -1, launch = -1, ncls = 0;
      expect("hsgn_autotune", hsgn_autotune(c, 2, tms, &kept), HSGN_OK, c);
      expect("hsgn_autotune_launch", hsgn_autotune_launch(c, 2, lms, &launch), HSGN_OK, c);
      std::vector<int32_t> cls(ni), keys(64 * 4), kept_c(64);
      std::vector<double> cms(64 * 3);
      expect("hsgn_autotune_classes",
             hsgn_autotune_classes(c, 2, 64, &ncls, cls.data(), keys.data(), cms.data(),
                                   kept_c.data(), whole),
             HSGN_OK, c);
      expect("hsgn_autotune_classes (room for one)",
             hsgn_autotune_classes(c, 2, 1, &ncls, nullptr, nullptr, nullptr, nullptr, nullptr),
             HSGN_EINVAL, c);
    }
    expect("hsgn_set_halo_margin (tiny)", hsgn_set_halo_margin(c, 1e-4), HSGN_OK, c);
    hsgn_step(c, 1);
    const int rs = hsgn_status(c, flags.data());
    std::printf("%-40s rc=%d\n", "hsgn_status (short halos)", rs);
    expect("hsgn_set_state (again)", hsgn_set_state(c, gh, gq, gm, gW, gt), HSGN_OK, c);
    expect("hsgn_set_halo_retry", hsgn_set_halo_retry(c, 1), HSGN_OK, c);
    expect("hsgn_run (retrying)", hsgn_run(c, 5, 2), HSGN_OK, c);
    expect("hsgn_step (retrying)", hsgn_step(c, 3), HSGN_OK, c);
    std::vector<double> margins(ni, 0.0);
    int32_t retries = -1;
    expect("hsgn_halo_state", hsgn_halo_state(c, margins.data(), &retries), HSGN_OK, c);
    std::printf("%-40s margins %g .. %g, %d blocks run again\n", "",
                *std::min_element(margins.begin(), margins.end()),
                *std::max_element(margins.begin(), margins.end()), retries);
    expect("hsgn_status (after retries)", hsgn_status(c, flags.data()), HSGN_OK, c);
    expect("hsgn_set_halo_retry (bad)", hsgn_set_halo_retry(c, 2), HSGN_EINVAL, c);
    expect("hsgn_set_halo_retry (off)", hsgn_set_halo_retry(c, 0), HSGN_OK, c);
    expect("hsgn_set_halo_margin (bad)", hsgn_set_halo_margin(c, -1.0), HSGN_EINVAL, c);
    expect("hsgn_set_halo_margin (default)", hsgn_set_halo_margin(c, 2.0), HSGN_OK, c);
  }
  expect("hsgn_set_solver (bad)", hsgn_set_solver(c, 7), HSGN_EINVAL, c);
  hsgn_destroy(c);
  for (double* p : {db, dh, dq, gh, gq, gm, gW, gt, gdt}) (void)hipFree(p);
}

void run_adjoint() {
  std::printf("== adjoint\n");
  Batch B = batch({300, 1001, 5000}, 2, HSGN_SCHEME_SEMI_IMPLICIT, true);
  for (auto& p : B.prm) p.dt_fixed = 0.01;
  const int ni = (int)B.prm.size(), ng = 3, nsteps = 7;
  double *db = dev(B.b), *dz = nullptr;
  std::vector<double> zeta(B.h.size());
  for (size_t i = 0; i < zeta.size(); ++i) zeta[i] = B.h[i] + B.b[i];
  dz = dev(zeta);
  std::vector<double> tg((size_t)ni * nsteps * ng, 0.4);
  double* dtg = dev(tg);
  std::vector<int32_t> gauge = {10, 20, 30, 100, 500, 900, 7, 2500, 4999};
  int32_t* dg = nullptr;
  hip_or_die(hipMalloc(&dg, gauge.size() * sizeof(int32_t)), "hipMalloc");
  hip_or_die(hipMemcpy(dg, gauge.data(), gauge.size() * sizeof(int32_t), hipMemcpyHostToDevice),
             "hipMemcpy");
  std::vector<double> zero(B.h.size(), 0.0), zi(ni, 0.0);
  double *dl = dev(zi), *gz = dev(zero), *gb = dev(zero);
  hsgn_ctx* c = nullptr;
  expect("hsgn_init (adjoint)", hsgn_init(&c, ni, B.off.data(), B.prm.data(), db, nullptr), HSGN_OK);
  if (!c) return;
  for (int64_t tb : {(int64_t)-1, (int64_t)0}) {
    expect("hsgn_set_adjoint_tape_bytes", hsgn_set_adjoint_tape_bytes(c, tb), HSGN_OK, c);
    for (int K : {2, 3, 7, 50}) {
      char what[64];
      std::snprintf(what, sizeof what, "hsgn_adjoint (K = %d, tape %lld)", K, (long long)tb);
      expect(what, hsgn_adjoint(c, nsteps, K, ng, dg, dtg, dz, dl, gz, gb), HSGN_OK, c);
    }
  }
  expect("hsgn_adjoint (loss only)", hsgn_adjoint(c, nsteps, 3, ng, dg, dtg, dz, dl, nullptr, nullptr),
         HSGN_OK, c);
  expect("hsgn_adjoint (bad K)", hsgn_adjoint(c, nsteps, 0, ng, dg, dtg, dz, dl, gz, gb),
         HSGN_EINVAL, c);
  hsgn_destroy(c);
  for (double* p : {db, dz, dtg, dl, gz, gb}) (void)hipFree(p);
  (void)hipFree(dg);
}

void run_noalloc() {
  std::printf("== noalloc\n");
  Batch B = batch({700, 3000, 9000}, 2, HSGN_SCHEME_SEMI_IMPLICIT, true);
  double *db = dev(B.b), *dh = dev(B.h), *dq = dev(B.q);
  std::vector<double> hm(B.h.size()), zero(B.h.size(), 0.0), zi(B.prm.size(), 0.0);
  for (size_t i = 0; i < hm.size(); ++i) hm[i] = B.h[i] * B.h[i];
  double *dm = dev(hm), *dW = dev(zero), *dt = dev(zi);
  std::vector<int32_t> flags(B.prm.size());
  char msg[HSGN_MSG_LEN];
  for (int32_t s : {HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT, HSGN_SOLVER_AUTO_SMALL})
    expect("hsgn_step_noalloc",
           hsgn_step_noalloc((int32_t)B.prm.size(), B.off.data(), B.prm.data(), db, dh, dq, dm, dW,
                             dt, 2, s, nullptr, flags.data(), msg),
           HSGN_OK);
  for (double* p : {db, dh, dq, dm, dW, dt}) (void)hipFree(p);
}

void run_invalid() {
  std::printf("== invalid input\n");
  hsgn_ctx* c = nullptr;
  int64_t off[3] = {0, 8, 11};
  hsgn_params p[2] = {params(1, 0, 2, 0, 100.0, 0.1), params(1, 0, 2, 0, 100.0, 0.1)};
  expect("hsgn_init (3 cells)", hsgn_init(&c, 2, off, p, nullptr, nullptr), HSGN_EINVAL);
  p[1].order = 1;
  off[2] = 16;
  expect("hsgn_init (orders differ)", hsgn_init(&c, 2, off, p, nullptr, nullptr), HSGN_EINVAL);
  expect("hsgn_step (null)", hsgn_step(nullptr, 1), HSGN_EINVAL);
  std::printf("last error of no context: \"%s\"\n", hsgn_last_error(nullptr));
  std::fflush(stdout);
}

}  // namespace

int main() {
  std::printf("%s\n", hsgn_version());
  run_invalid();
  run_context("semi-implicit, bed, mixed sizes",
              batch({4, 7, 513, 2047, 2048, 2049, 4097, 9000}, 2, HSGN_SCHEME_SEMI_IMPLICIT, true),
              true);
  run_context("first order", batch({5, 700, 5000}, 1, HSGN_SCHEME_SEMI_IMPLICIT, true), false);
  run_context("explicit", batch({4, 1023, 1025, 6000}, 2, HSGN_SCHEME_EXPLICIT, false), false);
  run_context("SGN", batch({4, 1023, 4096, 4097, 9000}, 2, HSGN_SCHEME_SGN, false), false);
  run_adjoint();
  run_noalloc();
  std::printf("%s\n", failures ? "FAILED" : "all calls returned as expected");
  return failures ? 1 : 0;
}

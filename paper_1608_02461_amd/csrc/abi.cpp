// extern "C" entry points of libhfmm.so (declared in include/hfmm.h).
// Every call converts C++ exceptions into an hfmm_status and a thread-local
// message; nothing throws across the interface.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "handles.h"
#include "solver.h"

namespace {
thread_local std::string g_last_error;
}

namespace hfmm {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace hfmm

extern "C" {

const char* hfmm_last_error(void) { return g_last_error.c_str(); }

int32_t hfmm_version(void) { return 100; }

hfmm_status hfmm_build_tree(const double* d_xy, int64_t n, double x0, double y0, double side, int32_t leaf_size,
                            hipStream_t stream, hfmm_tree* out) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(out != nullptr, "build_tree: out is NULL");
  *out = nullptr;
  auto h = std::make_unique<hfmm_tree_s>();
  h->t = hfmm::build_tree(d_xy, n, x0, y0, side, leaf_size, stream);
  *out = h.release();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tree_info(hfmm_tree t, int32_t* levels, int64_t* n_points, int64_t* n_leaves,
                           int32_t* max_leaf_count) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "tree_info: NULL tree");
  if (levels) *levels = t->t->L;
  if (n_points) *n_points = t->t->n;
  if (n_leaves) *n_leaves = t->t->nleaves;
  if (max_leaf_count) *max_leaf_count = t->t->max_leaf;
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tree_export(hfmm_tree t, int32_t* d_perm, int32_t* d_leaf_off, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "tree_export: NULL tree");
  const hfmm::Tree& tr = *t->t;
  if (d_perm) HFMM_HIP(hipMemcpyAsync(d_perm, tr.perm.p, tr.n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
  if (d_leaf_off)
    HFMM_HIP(hipMemcpyAsync(d_leaf_off, tr.leaf_off.p, (tr.nleaves + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice,
                            stream));
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tree_destroy(hfmm_tree t) {
  HFMM_GUARD_BEGIN
  delete t;
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_fmm_apply(hfmm_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q, void* d_phi,
                           int32_t nrhs, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "fmm_apply: NULL tree");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, "fmm_apply: unknown precision");
  HFMM_REQUIRE(nrhs >= 1 && nrhs <= 1024, "fmm_apply: nrhs must be in [1, 1024]");
  HFMM_REQUIRE(std::isfinite(k) && k > 0, "fmm_apply: k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 40, "fmm_apply: p must be in [1, 40]");
  HFMM_REQUIRE(d_q != nullptr && d_phi != nullptr, "fmm_apply: NULL array");
  if (prec == HFMM_FP64)
    hfmm::fmm_apply<double>(*t->t, k, p, static_cast<const double2*>(d_q), static_cast<double2*>(d_phi), nrhs,
                            stream);
  else
    hfmm::fmm_apply<float>(*t->t, k, p, static_cast<const float2*>(d_q), static_cast<float2*>(d_phi), nrhs, stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tree_set_options(hfmm_tree t, int32_t m2l_valu, int32_t autotune) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "tree_set_options: NULL tree");
  HFMM_REQUIRE((m2l_valu == 0 || m2l_valu == 1) && (autotune == 0 || autotune == 1),
               "tree_set_options: options must be 0 or 1");
  hfmm::Tree& tr = *t->t;
  if (tr.side) HFMM_HIP(hipStreamSynchronize(tr.side));
  tr.m2l_valu = m2l_valu != 0;
  tr.autotune = autotune != 0;
  tr.plans.clear();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tree_set_m2l_input_rounding(hfmm_tree t, int32_t mode) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "tree_set_m2l_input_rounding: NULL tree");
  HFMM_REQUIRE(mode >= 0 && mode <= 2, "tree_set_m2l_input_rounding: mode must be 0, 1 or 2");
  hfmm::Tree& tr = *t->t;
  if (tr.side) HFMM_HIP(hipStreamSynchronize(tr.side));
  HFMM_HIP(hipDeviceSynchronize());
  tr.m2l_round = mode;
  tr.plans.clear();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_fmm_apply_dipole(hfmm_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                                  const double* d_normals, void* d_phi, int32_t nrhs, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "fmm_apply_dipole: NULL tree");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, "fmm_apply_dipole: unknown precision");
  HFMM_REQUIRE(nrhs >= 1 && nrhs <= 1024, "fmm_apply_dipole: nrhs must be in [1, 1024]");
  HFMM_REQUIRE(std::isfinite(k) && k > 0, "fmm_apply_dipole: k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 40, "fmm_apply_dipole: p must be in [1, 40]");
  HFMM_REQUIRE(d_q != nullptr && d_phi != nullptr && d_normals != nullptr, "fmm_apply_dipole: NULL array");
  if (prec == HFMM_FP64)
    hfmm::fmm_apply_dipole<double>(*t->t, k, p, static_cast<const double2*>(d_q), d_normals,
                                   static_cast<double2*>(d_phi), nrhs, stream);
  else
    hfmm::fmm_apply_dipole<float>(*t->t, k, p, static_cast<const float2*>(d_q), d_normals,
                                  static_cast<float2*>(d_phi), nrhs, stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tune_cache_save(const char* path) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(path != nullptr, "tune_cache_save: NULL path");
  hfmm::tune_cache_save(path);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_tune_cache_load(const char* path, int32_t* n_loaded) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(path != nullptr, "tune_cache_load: NULL path");
  const int n = hfmm::tune_cache_load(path);
  if (n_loaded) *n_loaded = n;
  return HFMM_OK;
  HFMM_GUARD_END
}

int32_t hfmm_tune_cache_size(void) { return hfmm::tune_cache_size(); }

hfmm_status hfmm_tune_cache_clear(void) {
  HFMM_GUARD_BEGIN
  hfmm::tune_cache_clear();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_fmm_apply_timed(hfmm_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                                 void* d_phi, int32_t nrhs, float* ms_stages, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "fmm_apply_timed: NULL tree");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, "fmm_apply_timed: unknown precision");
  HFMM_REQUIRE(nrhs >= 1 && nrhs <= 1024, "fmm_apply_timed: nrhs must be in [1, 1024]");
  HFMM_REQUIRE(d_q != nullptr && d_phi != nullptr && ms_stages != nullptr, "fmm_apply_timed: NULL array");
  hfmm::StageTimer tm;
  if (prec == HFMM_FP64)
    hfmm::fmm_apply<double>(*t->t, k, p, static_cast<const double2*>(d_q), static_cast<double2*>(d_phi), nrhs,
                            stream, &tm);
  else
    hfmm::fmm_apply<float>(*t->t, k, p, static_cast<const float2*>(d_q), static_cast<float2*>(d_phi), nrhs, stream,
                           &tm);
  tm.collect(ms_stages, 9);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_fmm_plan_info(hfmm_tree t, double k, int32_t p, hfmm_precision prec, int32_t* orders,
                               int32_t* near_deg, int32_t* lanes_per_target, int64_t* pairs) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "fmm_plan_info: NULL tree");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, "fmm_plan_info: unknown precision");
  hfmm::Tree& tr = *t->t;
  auto fill = [&](auto& pl) {
    if (orders)
      for (int l = 0; l <= tr.L; ++l) orders[l] = pl.lv[l].p;
    if (near_deg) *near_deg = pl.near_fast ? pl.poly.deg : 0;
    if (lanes_per_target) *lanes_per_target = pl.G[0];
  };
  if (prec == HFMM_FP64)
    fill(hfmm::get_plan<double>(tr, k, p));
  else
    fill(hfmm::get_plan<float>(tr, k, p));
  if (pairs) {
    const int nb = 1 << tr.L;
    int64_t s = 0;
    for (int64_t b = 0; b < tr.nleaves; ++b) {
      const int64_t cnt = tr.leaf_off_h[b + 1] - tr.leaf_off_h[b];
      if (!cnt) continue;
      int bx, by;
      hfmm::demorton((uint32_t)b, bx, by);
      int64_t src = 0;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy) {
          const int sx = bx + dx, sy = by + dy;
          if (sx < 0 || sy < 0 || sx >= nb || sy >= nb) continue;
          const uint32_t sl = hfmm::morton((uint32_t)sx, (uint32_t)sy);
          src += tr.leaf_off_h[sl + 1] - tr.leaf_off_h[sl];
        }
      s += cnt * (src - 1);
    }
    *pairs = s;
  }
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_fd_helmholtz_matvec(int32_t n, double h, const double* d_k2, double k2_const, const double* d_x,
                                     double* d_y, int32_t nrhs, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(d_k2 != nullptr || std::isfinite(k2_const), "fd_matvec: k2_const must be finite");
  hfmm::fd_matvec(n, h, d_k2, k2_const, reinterpret_cast<const double2*>(d_x), reinterpret_cast<double2*>(d_y), nrhs,
                  stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_create(int32_t n, double h, const double* d_k2, double k2_const, double k0, int32_t p,
                               int32_t leaf_size, hfmm_precision precond_prec, int32_t nrhs, hipStream_t stream,
                               hfmm_solver* out) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(out != nullptr, "solver_create: out is NULL");
  *out = nullptr;
  HFMM_REQUIRE(precond_prec == HFMM_FP64 || precond_prec == HFMM_FP32, "solver_create: unknown precision");
  auto hs = std::make_unique<hfmm_solver_s>();
  hs->s = hfmm::solver_create(n, h, d_k2, k2_const, k0, p, leaf_size, precond_prec == HFMM_FP32, nrhs, stream);
  *out = hs.release();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_matched_wavenumber(double k, double h, double* k0) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(k0 != nullptr, "matched_wavenumber: k0 is NULL");
  HFMM_REQUIRE(std::isfinite(k) && std::isfinite(h) && k > 0 && h > 0 && k * h < 2.0,
               "matched_wavenumber: need k > 0, h > 0 and k h < 2");
  const double axis = 2.0 / h * std::asin(k * h / 2.0);
  const double diag = 2.0 * std::sqrt(2.0) / h * std::asin(k * h / (2.0 * std::sqrt(2.0)));
  *k0 = 0.5 * (axis + diag);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_set_k2(hfmm_solver s, const double* d_k2, double k2_const, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "set_k2: NULL solver");
  hfmm::solver_set_k2(*s->s, d_k2, k2_const, stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_set_k2_blocks(hfmm_solver s, const double* d_kb, int32_t nb, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "set_k2_blocks: NULL solver");
  hfmm::solver_set_k2_blocks(*s->s, d_kb, nb, stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_k2_gradient(int32_t n, const double* d_u, const double* d_mu, int32_t nb, double* d_grad,
                             hipStream_t stream) {
  HFMM_GUARD_BEGIN
  hfmm::k2_gradient(n, reinterpret_cast<const double2*>(d_u), reinterpret_cast<const double2*>(d_mu), nb, d_grad,
                    stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_dirichlet_apply(hfmm_solver s, const double* d_f, const double* d_g, double* d_u, int32_t nrhs,
                                 hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "dirichlet_apply: NULL solver");
  HFMM_REQUIRE(nrhs == s->s->nrhs, "dirichlet_apply: nrhs differs from the solver's");
  hfmm::dirichlet_apply(*s->s, reinterpret_cast<const double2*>(d_f), reinterpret_cast<const double2*>(d_g),
                        reinterpret_cast<double2*>(d_u), stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_boundary_nodes(hfmm_solver s, double* d_xy, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "solver_boundary_nodes: NULL solver");
  HFMM_REQUIRE(d_xy != nullptr, "solver_boundary_nodes: NULL array");
  const hfmm::Solver& sv = *s->s;
  std::vector<double> xy(2 * sv.ng);
  const int n = sv.n;
  for (int m = 0; m <= n; ++m) {
    const double t = (m + 0.5) * sv.h;
    const double pts[4][2] = {{t, 0.0}, {1.0, t}, {t, 1.0}, {0.0, t}};
    for (int side = 0; side < 4; ++side) {
      xy[2 * (side * (n + 1) + m)] = pts[side][0];
      xy[2 * (side * (n + 1) + m) + 1] = pts[side][1];
    }
  }
  HFMM_HIP(hipMemcpyAsync(d_xy, xy.data(), xy.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HFMM_HIP(hipStreamSynchronize(stream));  // the host buffer goes out of scope
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_bicgstab_solve(hfmm_solver s, const double* d_b, double* d_x, int32_t maxit, double rtol,
                                hfmm_solve_info* info, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "bicgstab_solve: NULL solver");
  return hfmm::bicgstab(*s->s, reinterpret_cast<const double2*>(d_b), reinterpret_cast<double2*>(d_x), maxit, rtol,
                        info, stream);
  HFMM_GUARD_END
}

hfmm_status hfmm_precond_apply(hfmm_solver s, const double* d_r, double* d_z, int32_t nrhs, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "precond_apply: NULL solver");
  HFMM_REQUIRE(nrhs == s->s->nrhs, "precond_apply: nrhs differs from the solver's");
  HFMM_REQUIRE(d_r != nullptr && d_z != nullptr && d_r != d_z, "precond_apply: NULL or aliased arrays");
  hfmm::Solver& sv = *s->s;
  hfmm::precond_apply(sv, reinterpret_cast<const double2*>(d_r), sv.nn, reinterpret_cast<double2*>(d_z), sv.nn,
                      nullptr, nullptr, stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_fgmres_solve(hfmm_solver s, const double* d_b, double* d_x, int32_t restart, int32_t maxit,
                              double rtol, int32_t transpose, hfmm_solve_info* info, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "fgmres_solve: NULL solver");
  HFMM_REQUIRE(transpose == 0 || transpose == 1, "fgmres_solve: transpose must be 0 or 1");
  // A^T = A for the FD operator with a real k^2 field, and M^{-1} is complex
  // symmetric, so the transposed solve is the same iteration.
  hfmm::Solver* sp = s->s.get();
  const double2* b = reinterpret_cast<const double2*>(d_b);
  double2* x = reinterpret_cast<double2*>(d_x);
  return hfmm::fgmres(&sp, 1, &b, &x, restart, maxit, rtol, false, info, stream);
  HFMM_GUARD_END
}

hfmm_status hfmm_fgmres_solve_batched(hfmm_solver* s, int32_t nprob, const double* const* d_b, double* const* d_x,
                                      int32_t restart, int32_t maxit, double rtol, int32_t use_graph,
                                      hfmm_solve_info* info, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && d_b != nullptr && d_x != nullptr, "solve_batched: NULL array");
  HFMM_REQUIRE(nprob >= 1, "solve_batched: nprob must be >= 1");
  std::vector<hfmm::Solver*> sp(nprob);
  std::vector<const double2*> b(nprob);
  std::vector<double2*> x(nprob);
  for (int i = 0; i < nprob; ++i) {
    HFMM_REQUIRE(s[i] != nullptr && s[i]->s, "solve_batched: NULL solver");
    for (int j = 0; j < i; ++j) HFMM_REQUIRE(s[j] != s[i], "solve_batched: a solver appears twice");
    sp[i] = s[i]->s.get();
    b[i] = reinterpret_cast<const double2*>(d_b[i]);
    x[i] = reinterpret_cast<double2*>(d_x[i]);
  }
  hipStream_t st = stream;
  hipStream_t own = nullptr;
  if (use_graph && st == nullptr) {  // the legacy default stream cannot be captured
    // work the caller queued on the default stream (its b and x) must be done
    // first: a non-blocking stream is not ordered after it
    HFMM_HIP(hipStreamSynchronize(nullptr));
    HFMM_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    st = own;
  }
  hfmm_status r;
  try {
    r = hfmm::fgmres(sp.data(), nprob, b.data(), x.data(), restart, maxit, rtol, use_graph != 0, info, st);
  } catch (...) {
    if (own) {
      (void)hipStreamSynchronize(own);
      (void)hipStreamDestroy(own);
    }
    throw;
  }
  if (own) {
    HFMM_HIP(hipStreamSynchronize(own));
    HFMM_HIP(hipStreamDestroy(own));
  }
  return r;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_info(hfmm_solver s, int32_t* n_gamma, double* cond_S, int32_t* levels, int32_t* leaf_size) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "solver_info: NULL solver");
  if (n_gamma) *n_gamma = (int32_t)s->s->ng;
  if (cond_S) *cond_S = s->s->condS;
  if (levels) *levels = s->s->tree->L;
  if (leaf_size) *leaf_size = s->s->leaf;
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_set_m2l_input_rounding(hfmm_solver s, int32_t mode) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "solver_set_m2l_input_rounding: NULL solver");
  HFMM_REQUIRE(mode >= 0 && mode <= 2, "solver_set_m2l_input_rounding: mode must be 0, 1 or 2");
  hfmm::Solver& sv = *s->s;
  hfmm::Tree& tr = *sv.tree;
  if (tr.side) HFMM_HIP(hipStreamSynchronize(tr.side));
  HFMM_HIP(hipDeviceSynchronize());
  sv.drop_step_graph();
  tr.m2l_round = mode;
  tr.plans.clear();
  if (sv.fp32)
    (void)hfmm::get_plan<float>(tr, sv.k0, sv.p);
  else
    (void)hfmm::get_plan<double>(tr, sv.k0, sv.p);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm_solver_destroy(hfmm_solver s) {
  HFMM_GUARD_BEGIN
  delete s;
  return HFMM_OK;
  HFMM_GUARD_END
}

// ------------------------------------------------------------------ 3-D oct-tree FMM
hfmm_status hfmm3_build_tree(const double* d_xyz, int64_t n, double x0, double y0, double z0, double side,
                             int32_t leaf_size, hipStream_t stream, hfmm3_tree* out) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(out != nullptr, "build_tree3: out is NULL");
  *out = nullptr;
  auto h = std::make_unique<hfmm3_tree_s>();
  h->t = hfmm::build_tree3(d_xyz, n, x0, y0, z0, side, leaf_size, stream);
  *out = h.release();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_tree_info(hfmm3_tree t, int32_t* levels, int64_t* n_points, int64_t* n_leaves,
                            int32_t* max_leaf_count) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "tree3_info: NULL tree");
  if (levels) *levels = t->t->L;
  if (n_points) *n_points = t->t->n;
  if (n_leaves) *n_leaves = t->t->nleaves;
  if (max_leaf_count) *max_leaf_count = t->t->max_leaf;
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_tree_destroy(hfmm3_tree t) {
  HFMM_GUARD_BEGIN
  delete t;
  return HFMM_OK;
  HFMM_GUARD_END
}

static void fmm3_check(hfmm3_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q, const void* d_phi,
                       const char* who) {
  HFMM_REQUIRE(t != nullptr && t->t, std::string(who) + ": NULL tree");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, std::string(who) + ": unknown precision");
  HFMM_REQUIRE(std::isfinite(k) && k > 0, std::string(who) + ": k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 20, std::string(who) + ": p must be in [1, 20]");
  HFMM_REQUIRE(d_q != nullptr && d_phi != nullptr, std::string(who) + ": NULL array");
}

hfmm_status hfmm3_fmm_apply(hfmm3_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                            void* d_phi, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  fmm3_check(t, k, p, prec, d_q, d_phi, "fmm3_apply");
  if (prec == HFMM_FP64)
    hfmm::fmm3_apply<double>(*t->t, k, p, static_cast<const double2*>(d_q), static_cast<double2*>(d_phi), stream,
                             nullptr);
  else
    hfmm::fmm3_apply<float>(*t->t, k, p, static_cast<const float2*>(d_q), static_cast<float2*>(d_phi), stream,
                            nullptr);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_fmm_apply_timed(hfmm3_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                                  void* d_phi, float* ms_stages, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  fmm3_check(t, k, p, prec, d_q, d_phi, "fmm3_apply_timed");
  HFMM_REQUIRE(ms_stages != nullptr, "fmm3_apply_timed: ms_stages is NULL");
  if (prec == HFMM_FP64)
    hfmm::fmm3_apply<double>(*t->t, k, p, static_cast<const double2*>(d_q), static_cast<double2*>(d_phi), stream,
                             ms_stages);
  else
    hfmm::fmm3_apply<float>(*t->t, k, p, static_cast<const float2*>(d_q), static_cast<float2*>(d_phi), stream,
                            ms_stages);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_fmm_orders(hfmm3_tree t, double k, int32_t p, int32_t* orders) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "fmm3_orders: NULL tree");
  HFMM_REQUIRE(orders != nullptr, "fmm3_orders: orders is NULL");
  const std::vector<int> o = hfmm::fmm3_orders(*t->t, k, p);
  for (size_t l = 0; l < o.size(); ++l) orders[l] = o[l];
  return HFMM_OK;
  HFMM_GUARD_END
}

// ------------------------------------------------------------------ 3-D model problem
hfmm_status hfmm3_fd_matvec(int32_t n, double k2, const double* d_x, double* d_y, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(n >= 1 && n <= 1024, "fd3_matvec: n must be in [1, 1024]");
  HFMM_REQUIRE(std::isfinite(k2), "fd3_matvec: k2 must be finite");
  HFMM_REQUIRE(d_x != nullptr && d_y != nullptr, "fd3_matvec: NULL array");
  HFMM_REQUIRE(d_x != d_y, "fd3_matvec: x and y must not alias");
  hfmm::fd3_apply(n, k2, reinterpret_cast<const double2*>(d_x), reinterpret_cast<double2*>(d_y), nullptr, stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_solver_create(int32_t n, double k, int32_t p, int32_t leaf_size, hfmm_precision precond_prec,
                                hipStream_t stream, hfmm3_solver* out) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(out != nullptr, "solver3_create: out is NULL");
  *out = nullptr;
  auto h = std::make_unique<hfmm3_solver_s>();
  h->s = std::make_unique<hfmm::Solver3>(n, k, p, leaf_size, (int)precond_prec, stream);
  *out = h.release();
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_precond_apply(hfmm3_solver s, const double* d_r, double* d_z, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "precond3_apply: NULL solver");
  HFMM_REQUIRE(d_r != nullptr && d_z != nullptr, "precond3_apply: NULL array");
  HFMM_REQUIRE(d_r != d_z, "precond3_apply: r and z must not alias");
  s->s->precond(reinterpret_cast<const double2*>(d_r), reinterpret_cast<double2*>(d_z), stream);
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_fgmres_solve(hfmm3_solver s, const double* d_b, double* d_x, int32_t restart, int32_t maxit,
                               double rtol, hfmm_solve_info* info, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "fgmres3: NULL solver");
  const hfmm::Solve3Result r = s->s->fgmres(reinterpret_cast<const double2*>(d_b), reinterpret_cast<double2*>(d_x),
                                            restart, maxit, rtol, stream);
  if (info) {
    *info = hfmm_solve_info{};
    info->iters = r.iters;
    info->restarts = r.restarts;
    info->converged = r.converged ? 1 : 0;
    info->rel_res_true = r.rel_res_true;
    info->rel_res_est = r.rel_res_est;
    info->nrhs = 1;
    info->ms_precond = r.ms_precond;
    info->ms_total = r.ms_total;
    info->ms_krylov = r.ms_total - r.ms_precond;
    info->ms_setup = s->s->ms_setup;
  }
  if (r.numeric) {
    hfmm::set_last_error("fgmres3: NaN or Inf met");
    return HFMM_ERR_NUMERIC;
  }
  return r.converged ? HFMM_OK : HFMM_NOT_CONVERGED;
  HFMM_GUARD_END
}

hfmm_status hfmm3_solver_info(hfmm3_solver s, double* self_term, int32_t* levels, double* ms_setup) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(s != nullptr && s->s, "solver3_info: NULL solver");
  if (self_term) {
    self_term[0] = s->s->cself.real();
    self_term[1] = s->s->cself.imag();
  }
  if (levels) *levels = s->s->tree->L;
  if (ms_setup) *ms_setup = s->s->ms_setup;
  return HFMM_OK;
  HFMM_GUARD_END
}

hfmm_status hfmm3_solver_destroy(hfmm3_solver s) {
  HFMM_GUARD_BEGIN
  delete s;
  return HFMM_OK;
  HFMM_GUARD_END
}

}  // extern "C"

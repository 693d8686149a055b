// The 3-D model problem (Sec. 7, eq. helm3) on a 7-point grid with the
// oct-tree FMM volume potential as the FGMRES preconditioner.
#pragma once

#include <complex>
#include <memory>

#include "fmm3.h"

namespace hfmm {

struct Solve3Result {
  int iters = 0, restarts = 0;
  bool converged = false, numeric = false;
  double rel_res_true = 0, rel_res_est = 0, ms_precond = 0, ms_total = 0;
};

// Integral of exp(i k r)/(4 pi r) over a cube of side h about its centre.
std::complex<double> cell_self_term3(double k, double h);

// y = (-Laplace_h - k^2) x on n^3 nodes (zero ghost values), or y = b - A x
// when b is given; complex128, x fastest.  Async on st.
void fd3_apply(int n, double k2, const double2* x, double2* y, const double2* b, hipStream_t st);

struct Solver3 {
  int n = 0, p = 0, prec = 0;
  double k = 0, h = 0, ms_setup = 0;
  int64_t N = 0;
  std::unique_ptr<Tree3> tree;
  std::complex<double> cself;
  DevBuf<double2> V, Z, w, q64, phi64, cdev;
  DevBuf<float2> q32, phi32;
  DevBuf<double> part;

  Solver3(int n, double k, int p, int leaf, int prec, hipStream_t st);
  Solver3(const Solver3&) = delete;
  Solver3& operator=(const Solver3&) = delete;
  // z = h^3 FMM(r) + c_self r (the FMM in the solver's precision)
  void precond(const double2* r, double2* z, hipStream_t st);
  // right-preconditioned FGMRES(m); x holds x0 on entry.  Synchronises st.
  Solve3Result fgmres(const double2* b, double2* x, int m, int maxit, double rtol, hipStream_t st);

 private:
  void mdot(const double2* V, int nt, const double2* x, std::complex<double>* out, hipStream_t st);
  void msub(const double2* V, int nt, const std::complex<double>* c, double2* x, hipStream_t st);
  double norm(const double2* x, hipStream_t st);
};

}  // namespace hfmm

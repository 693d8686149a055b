// FD Helmholtz operator, FMM-BEM preconditioner and device FGMRES.
#pragma once

#include <complex>

#include "fmm.h"

namespace hfmm {

void fd_matvec(int n, double h, const double* d_k2, double k2c, const double2* x, double2* y, int nrhs,
               hipStream_t st);

struct Solver {
  int n = 0;
  double h = 0;
  int64_t nn = 0;   // interior unknowns n*n
  int64_t ng = 0;   // boundary elements 4(n+1)
  int nrhs = 1;
  double k0 = 0;
  int p = 0, leaf = 0;
  bool fp32 = false;
  DevBuf<double> k2;
  double k2c = 0;
  bool field = false;
  std::unique_ptr<Tree> tree;
  DevBuf<uint8_t> flags1, flags2;  // per-level source flags: interior / boundary sources
  DevBuf<float2> B32;              // -w S^{-1}, ng x ng row-major
  DevBuf<double2> B64;
  std::complex<double> svol;       // volume self term
  double condS = 0;
  // preconditioner scratch in sorted order (nrhs columns)
  DevBuf<float2> q1f, phif, q2f, vgf;
  DevBuf<double2> q1d, phid, q2d, vgd;
  // Krylov workspace
  int m = 0;
  int nblk = 0;
  DevBuf<double2> V, Z, H, sn, g, y, hcur, part;
  DevBuf<double> cs, bnorm, est, rn, npart;
  DevBuf<int> active, jj, iters, state;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  // one Arnoldi step captured into a graph (batched solve with graphs), kept
  // from one solve to the next while restart, maxit and rtol are the same;
  // every change to the solver drops it
  hipGraph_t step_graph = nullptr;
  hipGraphExec_t step_exec = nullptr;
  int step_m = 0, step_maxit = 0;
  double step_rtol = 0;
  void drop_step_graph();
  double ms_setup = 0;             // wall time of solver_create (ms)
  std::vector<std::pair<int, float>> leaf_ms;  // leaf-size candidates timed (leaf_size 0)
  // outward unit normals of the boundary elements at their sorted slots
  // (zero at interior nodes), for the double-layer pass
  DevBuf<float2> nrm32;
  DevBuf<double2> nrm64;
  // BiCGSTAB workspace: r, r^, p, v, s, t, p^, s^ (n*n x nrhs each) and scalars
  DevBuf<double2> bw;
  DevBuf<double2> bsc;
  DevBuf<double> bpart;
  DevBuf<int> bact;
  ~Solver();
};

std::unique_ptr<Solver> solver_create(int n, double h, const double* d_k2, double k2c, double k0, int p, int leaf,
                                      bool fp32, int nrhs, hipStream_t st);
void solver_set_k2(Solver& s, const double* d_k2, double k2c, hipStream_t st);
// z = M^{-1} r; r, z column stride rs, zs (complex elements).  j_from_state: when
// non-NULL, column c reads r + c*rs + state[0]*nn and writes z + c*zs + state[0]*nn.
void precond_apply(Solver& s, const double2* r, int64_t rs, double2* z, int64_t zs, const int* jstate,
                   const int* alive, hipStream_t st);
hfmm_status fgmres(Solver** s, int nprob, const double2* const* b, double2* const* x, int m, int maxit, double rtol,
                   bool use_graph, hfmm_solve_info* info, hipStream_t st);

// u = the boundary-element solution with source f and Dirichlet data g at
// the element midpoints (Sec. 5.2, boundary and interior equations with the
// double-layer and 1/2 delta terms).  f, u: n*n x nrhs; g: 4(n+1) x nrhs.
void dirichlet_apply(Solver& s, const double2* f, const double2* g, double2* u, hipStream_t st);

// k^2 constant on nb x nb blocks of (n/nb)^2 nodes; kb row-major, block rows follow y.
void solver_set_k2_blocks(Solver& s, const double* kb, int nb, hipStream_t st);

// grad[b] = sum over the nodes x of block b of Re(conj(mu_x) u_x) (n/nb nodes a side).
void k2_gradient(int n, const double2* u, const double2* mu, int nb, double* grad, hipStream_t st);

// Right-preconditioned BiCGSTAB (van der Vorst 1992) with the same operator
// and preconditioner; all FP64 on the device.
hfmm_status bicgstab(Solver& s, const double2* b, double2* x, int maxit, double rtol, hfmm_solve_info* info,
                     hipStream_t st);

}  // namespace hfmm

// The 3-D model problem of Sec. 7 (eq. helm3) on a 7-point finite-difference
// grid, solved by right-preconditioned FGMRES(m) (Sec. 3-4) with the 3-D FMM
// of the oct-tree as the preconditioner: the volume potential of the residual
// (Sec. 5, in 3-D, without the boundary-element correction of Sec. 5.2 for
// the cube's faces),
//   z_i = h^3 sum_{j != i} G(|x_i - x_j|) r_j + c_self r_i,  G = exp(i k r)/(4 pi r),
// c_self the integral of G over the node's cell.
//
// Layout: vectors are complex128, interleaved, nodes (i h, j h, l h) with
// h = 1/(n+1), x fastest; the oct-tree is built over the nodes in that order,
// so the FMM's caller order is the grid order.  The Krylov basis V ((m+1) N)
// and the preconditioned vectors Z (m N) live on the device; the Hessenberg
// matrix and the Givens rotations (at most m = 200) on the host.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "devutil.h"
#include "fmm3.h"
#include "solver3.h"
#include "special.h"

namespace hfmm {

namespace {

constexpr int kRedBlocks3 = 1024;  // blocks of the dot-product partial sums (4 per CU)
constexpr int kMaxDots3 = 8;       // dots per pass of the multi-dot kernel
constexpr int kMaxVecs3 = 208;     // V_0 .. V_m for m <= 200, in whole passes of 8

inline int nblk(int64_t n) { return (int)((n + 255) / 256); }

// y = (-Laplace_h - k^2) x, zero ghost values
__global__ void k3_fd(int n, double ih2, double k2, const double2* __restrict__ x, double2* __restrict__ y,
                      const double2* __restrict__ b) {
  const int64_t N = (int64_t)n * n * n;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g % n), j = (int)((g / n) % n), l = (int)(g / ((int64_t)n * n));
  const int64_t sy = n, sz = (int64_t)n * n;
  const double2 c = x[g];
  double re = 0, im = 0;
  if (i > 0) { re += x[g - 1].x; im += x[g - 1].y; }
  if (i < n - 1) { re += x[g + 1].x; im += x[g + 1].y; }
  if (j > 0) { re += x[g - sy].x; im += x[g - sy].y; }
  if (j < n - 1) { re += x[g + sy].x; im += x[g + sy].y; }
  if (l > 0) { re += x[g - sz].x; im += x[g - sz].y; }
  if (l < n - 1) { re += x[g + sz].x; im += x[g + sz].y; }
  double2 o;
  o.x = (6.0 * c.x - re) * ih2 - k2 * c.x;
  o.y = (6.0 * c.y - im) * ih2 - k2 * c.y;
  if (b) {  // residual b - A x
    o.x = b[g].x - o.x;
    o.y = b[g].y - o.y;
  }
  y[g] = o;
}

// partial sums of conj(V_t) . w for t < nt: part[(t * nb + block) * 2 + {re, im}]
__global__ __launch_bounds__(256) void k3_mdot(const double2* __restrict__ V, int64_t N, int nt,
                                               const double2* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[2][kMaxDots3][4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double sr[kMaxDots3], si[kMaxDots3];
#pragma unroll
  for (int t = 0; t < kMaxDots3; ++t) sr[t] = si[t] = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * 256 + tid; g < N; g += (int64_t)gridDim.x * 256) {
    const double2 b = w[g];
#pragma unroll
    for (int t = 0; t < kMaxDots3; ++t)
      if (t < nt) {
        const double2 a = V[t * N + g];
        sr[t] += a.x * b.x + a.y * b.y;
        si[t] += a.x * b.y - a.y * b.x;
      }
  }
#pragma unroll
  for (int t = 0; t < kMaxDots3; ++t) {
    double r = sr[t], i = si[t];
    for (int o = 32; o >= 1; o >>= 1) {
      r += __shfl_xor(r, o);
      i += __shfl_xor(i, o);
    }
    if (lane == 0) {
      red[0][t][wv] = r;
      red[1][t][wv] = i;
    }
  }
  __syncthreads();
  if (tid < nt) {
    const double r = red[0][tid][0] + red[0][tid][1] + red[0][tid][2] + red[0][tid][3];
    const double i = red[1][tid][0] + red[1][tid][1] + red[1][tid][2] + red[1][tid][3];
    part[((size_t)tid * gridDim.x + blockIdx.x) * 2] = r;
    part[((size_t)tid * gridDim.x + blockIdx.x) * 2 + 1] = i;
  }
}

// w -= sum_t V_t c_t (c on the device, complex)
__global__ void k3_msub(const double2* __restrict__ V, int64_t N, int nt, const double2* __restrict__ c,
                        double2* __restrict__ w) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double2 o = w[g];
  for (int t = 0; t < nt; ++t) {
    const double2 a = V[t * N + g], s = c[t];
    o.x -= a.x * s.x - a.y * s.y;
    o.y -= a.x * s.y + a.y * s.x;
  }
  w[g] = o;
}

// y = s x (real s)
__global__ void k3_scale(const double2* __restrict__ x, double s, int64_t N, double2* __restrict__ y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const double2 v = x[g];
  y[g] = make_double2(v.x * s, v.y * s);
}

// preconditioner staging: q = h^3 r in the FMM's precision
template <class T>
__global__ void k3_prec_in(const double2* __restrict__ r, double h3, int64_t N, cplx<T>* __restrict__ q) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  q[g] = mk<T>(T(r[g].x * h3), T(r[g].y * h3));
}
// z = phi + c_self r
template <class T>
__global__ void k3_prec_out(const cplx<T>* __restrict__ phi, const double2* __restrict__ r, double cr, double ci,
                            int64_t N, double2* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const double2 v = r[g];
  z[g] = make_double2((double)phi[g].x + cr * v.x - ci * v.y, (double)phi[g].y + cr * v.y + ci * v.x);
}

__global__ void k3_grid(int n, double h, double* __restrict__ xyz) {
  const int64_t N = (int64_t)n * n * n;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  xyz[3 * g] = (double)(g % n + 1) * h;
  xyz[3 * g + 1] = (double)((g / n) % n + 1) * h;
  xyz[3 * g + 2] = (double)(g / ((int64_t)n * n) + 1) * h;
}

}  // namespace

// Integral of exp(i k r)/(4 pi r) over the cube [-h/2, h/2]^3.  In spherical
// coordinates about the centre the radial integral is closed:
// int_0^R r exp(i k r) dr = R^2 sum_n (i k R)^n / (n! (n + 2)); over the
// face z = h/2, dOmega = (h/2) da db / R^3, R = |(a, b, h/2)|, so
//   c = 6/(4 pi) int_face (h/2) S(k R) / R da db,  S(x) = sum_n (i x)^n/(n! (n+2)),
// by Gauss-Legendre in a and b (the integrand is smooth on the face).
std::complex<double> cell_self_term3(double k, double h) {
  const int nq = 32;
  std::vector<double> xs, ws;
  gauss_legendre(nq, xs, ws);
  std::complex<double> acc = 0.0;
  for (int ia = 0; ia < nq; ++ia)
    for (int ib = 0; ib < nq; ++ib) {
      const double a = 0.5 * h * xs[ia], b = 0.5 * h * xs[ib];
      const double wgt = 0.25 * h * h * ws[ia] * ws[ib];
      const double R = std::sqrt(a * a + b * b + 0.25 * h * h);
      const double x = k * R;
      std::complex<double> S = 0.0, term = 1.0;  // term = (i x)^n / n!
      for (int m = 0; m < 200; ++m) {
        if (m > 0) term *= std::complex<double>(0.0, x) / double(m);
        S += term / double(m + 2);
        if (std::abs(term) < 1e-18 && m > 4) break;
      }
      acc += wgt * (0.5 * h) * S / R;
    }
  return 6.0 / (4.0 * 3.14159265358979323846) * acc;
}

void fd3_apply(int n, double k2, const double2* x, double2* y, const double2* b, hipStream_t st) {
  const double h = 1.0 / (n + 1);
  const int64_t N = (int64_t)n * n * n;
  k3_fd<<<nblk(N), 256, 0, st>>>(n, 1.0 / (h * h), k2, x, y, b);
  HFMM_LAUNCH_CHECK();
}

Solver3::Solver3(int n_, double k_, int p_, int leaf, int prec_, hipStream_t st)
    : n(n_), k(k_), p(p_), prec(prec_) {
  const auto t0 = std::chrono::steady_clock::now();
  HFMM_REQUIRE(n >= 2 && n <= 512, "solver3_create: n must be in [2, 512]");
  HFMM_REQUIRE(std::isfinite(k) && k > 0, "solver3_create: k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 20, "solver3_create: p must be in [1, 20]");
  HFMM_REQUIRE(leaf >= 1, "solver3_create: leaf_size must be >= 1");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, "solver3_create: unknown precision");
  h = 1.0 / (n + 1);
  N = (int64_t)n * n * n;
  DevBuf<double> xyz(3 * N);
  k3_grid<<<nblk(N), 256, 0, st>>>(n, h, xyz.p);
  HFMM_LAUNCH_CHECK();
  tree = build_tree3(xyz.p, N, 0.0, 0.0, 0.0, 1.0, leaf, st);
  HFMM_REQUIRE(tree->L >= 2, "solver3_create: the tree needs depth >= 2 (lower leaf_size)");
  cself = cell_self_term3(k, h);
  w.alloc(N);
  if (prec == HFMM_FP64) {
    q64.alloc(N);
    phi64.alloc(N);
  } else {
    q32.alloc(N);
    phi32.alloc(N);
  }
  part.alloc((size_t)kMaxVecs3 * kRedBlocks3 * 2);
  cdev.alloc(kMaxVecs3);
  // the plan (translation tables) now, so that a solve allocates nothing for it
  DevBuf<double2> r0(N), z0(N);
  HFMM_HIP(hipMemsetAsync(r0.p, 0, N * sizeof(double2), st));
  precond(r0.p, z0.p, st);
  HFMM_HIP(hipStreamSynchronize(st));
  ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void Solver3::precond(const double2* r, double2* z, hipStream_t st) {
  if (prec == HFMM_FP64) {
    k3_prec_in<double><<<nblk(N), 256, 0, st>>>(r, h * h * h, N, q64.p);
    HFMM_LAUNCH_CHECK();
    fmm3_apply<double>(*tree, k, p, q64.p, phi64.p, st, nullptr);
    k3_prec_out<double><<<nblk(N), 256, 0, st>>>(phi64.p, r, cself.real(), cself.imag(), N, z);
  } else {
    k3_prec_in<float><<<nblk(N), 256, 0, st>>>(r, h * h * h, N, q32.p);
    HFMM_LAUNCH_CHECK();
    fmm3_apply<float>(*tree, k, p, q32.p, phi32.p, st, nullptr);
    k3_prec_out<float><<<nblk(N), 256, 0, st>>>(phi32.p, r, cself.real(), cself.imag(), N, z);
  }
  HFMM_LAUNCH_CHECK();
}

// conj(V_t) . w for t < nt: every pass of 8 writes its own rows of partial
// sums, one copy back, summed on the host in a fixed order
void Solver3::mdot(const double2* V, int nt, const double2* x, std::complex<double>* out, hipStream_t st) {
  HFMM_REQUIRE(nt >= 1 && nt <= kMaxVecs3, "fgmres3: too many basis vectors");
  for (int t0 = 0; t0 < nt; t0 += kMaxDots3) {
    const int c = std::min(kMaxDots3, nt - t0);
    k3_mdot<<<kRedBlocks3, 256, 0, st>>>(V + t0 * N, N, c, x, part.p + (size_t)t0 * kRedBlocks3 * 2);
    HFMM_LAUNCH_CHECK();
  }
  std::vector<double> hp((size_t)nt * kRedBlocks3 * 2);
  HFMM_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HFMM_HIP(hipStreamSynchronize(st));
  for (int t = 0; t < nt; ++t) {
    double re = 0, im = 0;
    for (int b = 0; b < kRedBlocks3; ++b) {
      re += hp[((size_t)t * kRedBlocks3 + b) * 2];
      im += hp[((size_t)t * kRedBlocks3 + b) * 2 + 1];
    }
    out[t] = {re, im};
  }
}

// x -= sum_t V_t c_t: the nt coefficients go up in one copy, then passes of 8
void Solver3::msub(const double2* V, int nt, const std::complex<double>* c, double2* x, hipStream_t st) {
  HFMM_REQUIRE(nt >= 1 && nt <= kMaxVecs3, "fgmres3: too many basis vectors");
  HFMM_HIP(hipMemcpyAsync(cdev.p, c, nt * sizeof(double2), hipMemcpyHostToDevice, st));
  for (int t0 = 0; t0 < nt; t0 += kMaxDots3) {
    const int cn = std::min(kMaxDots3, nt - t0);
    k3_msub<<<nblk(N), 256, 0, st>>>(V + t0 * N, N, cn, cdev.p + t0, x);
    HFMM_LAUNCH_CHECK();
  }
  HFMM_HIP(hipStreamSynchronize(st));  // the host coefficients and cdev are reused
}

double Solver3::norm(const double2* x, hipStream_t st) {
  std::complex<double> d;
  mdot(x, 1, x, &d, st);
  return std::sqrt(std::max(0.0, d.real()));
}

Solve3Result Solver3::fgmres(const double2* b, double2* x, int m, int maxit, double rtol, hipStream_t st) {
  HFMM_REQUIRE(m >= 1 && m <= 200, "fgmres3: restart must be in [1, 200]");
  HFMM_REQUIRE(maxit >= 1, "fgmres3: maxit must be >= 1");
  HFMM_REQUIRE(rtol > 0 && std::isfinite(rtol), "fgmres3: rtol must be > 0");
  HFMM_REQUIRE(b != nullptr && x != nullptr, "fgmres3: NULL vector");
  const auto t0 = std::chrono::steady_clock::now();
  if (V.n < (size_t)(m + 1) * N) V.alloc((size_t)(m + 1) * N);
  if (Z.n < (size_t)m * N) Z.alloc((size_t)m * N);
  using C = std::complex<double>;
  Solve3Result res;
  const double bnorm = norm(b, st);
  if (!(bnorm > 0)) {
    HFMM_HIP(hipMemsetAsync(x, 0, N * sizeof(double2), st));
    HFMM_HIP(hipStreamSynchronize(st));
    res.converged = std::isfinite(bnorm);
    res.numeric = !std::isfinite(bnorm);
    return res;
  }
  std::vector<C> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), hcol(m + 1), h2(m + 1), y(m);
  double ms_prec = 0;
  for (;;) {
    fd3_apply(n, k * k, x, V.p, b, st);  // V_0 = b - A x
    const double beta = norm(V.p, st);
    res.rel_res_true = beta / bnorm;
    if (!std::isfinite(beta)) {
      res.numeric = true;
      break;
    }
    if (beta <= rtol * bnorm) {
      res.converged = true;
      break;
    }
    if (res.iters >= maxit) break;
    k3_scale<<<nblk(N), 256, 0, st>>>(V.p, 1.0 / beta, N, V.p);
    HFMM_LAUNCH_CHECK();
    std::fill(g.begin(), g.end(), C(0));
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double2* Vj = V.p + (size_t)j * N;
      double2* Zj = Z.p + (size_t)j * N;
      double2* Vn = V.p + (size_t)(j + 1) * N;
      const auto tp = std::chrono::steady_clock::now();
      precond(Vj, Zj, st);
      HFMM_HIP(hipStreamSynchronize(st));
      ms_prec += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
      fd3_apply(n, k * k, Zj, Vn, nullptr, st);
      // classical Gram-Schmidt, twice
      mdot(V.p, j + 1, Vn, hcol.data(), st);
      msub(V.p, j + 1, hcol.data(), Vn, st);
      mdot(V.p, j + 1, Vn, h2.data(), st);
      msub(V.p, j + 1, h2.data(), Vn, st);
      for (int t = 0; t <= j; ++t) hcol[t] += h2[t];
      const double hn = norm(Vn, st);
      hcol[j + 1] = hn;
      if (hn > 0) {
        k3_scale<<<nblk(N), 256, 0, st>>>(Vn, 1.0 / hn, N, Vn);
        HFMM_LAUNCH_CHECK();
      }
      // previous rotations, then a new one that zeroes hcol[j+1]
      for (int t = 0; t < j; ++t) {
        const C a = hcol[t], c2 = hcol[t + 1];
        hcol[t] = std::conj(cs[t]) * a + std::conj(sn[t]) * c2;
        hcol[t + 1] = -sn[t] * a + cs[t] * c2;
      }
      const double den = std::sqrt(std::norm(hcol[j]) + std::norm(hcol[j + 1]));
      if (den > 0) {
        cs[j] = hcol[j] / den;
        sn[j] = hcol[j + 1] / den;
      } else {
        cs[j] = 1.0;
        sn[j] = 0.0;
      }
      hcol[j] = den;
      hcol[j + 1] = 0.0;
      const C gj = g[j];
      g[j] = std::conj(cs[j]) * gj;
      g[j + 1] = -sn[j] * gj;
      for (int t = 0; t <= j; ++t) H[(size_t)t * m + j] = hcol[t];
      ++res.iters;
      jend = j + 1;
      res.rel_res_est = std::abs(g[j + 1]) / bnorm;
      if (std::abs(g[j + 1]) <= rtol * bnorm || res.iters >= maxit || !(hn > 0)) break;
    }
    // x += Z R^{-1} g
    for (int t = jend - 1; t >= 0; --t) {
      C s = g[t];
      for (int u = t + 1; u < jend; ++u) s -= H[(size_t)t * m + u] * y[u];
      y[t] = H[(size_t)t * m + t] != C(0) ? s / H[(size_t)t * m + t] : C(0);
    }
    std::vector<C> ny(jend);
    for (int t = 0; t < jend; ++t) ny[t] = -y[t];  // msub subtracts
    msub(Z.p, jend, ny.data(), x, st);
    ++res.restarts;
  }
  res.ms_precond = ms_prec;
  res.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return res;
}

}  // namespace hfmm

// Vector kernels of the start of preconditioned CG (§3
// eq:cg-energy-norm-error-reduction, stopping rule of §4.1) and of the shifted
// inverse iteration with B-normalisation (§2).  The CG iteration itself is
// fused into the stencil (direction update), the restriction (x and r update)
// and the extension (stopping test).  Scalars stay on the device: a kernel
// that needs a global sum adds the per-block partials of the kernel before it
// in a fixed order (Red), so no host round trip is needed inside an iteration
// and sums are deterministic.  After convergence or breakdown the state's
// `done` flag turns every later iteration kernel into a no-op, so the host can
// queue several iterations between checks.
#include "k_common.h"

namespace ddeig {

// Grid of a reducing elementwise kernel: two elements per thread, at most kMaxRed blocks.
int red_grid(long work) {
  const long b = (work + 2L * kBlock - 1) / (2L * kBlock);
  return (int)std::max<long>(1, std::min<long>(b, kMaxRed));
}

__global__ void k_resid_init(long n, const double* __restrict__ b, const double* __restrict__ q,
                             double* __restrict__ r, Red rr) {
  double acc = 0.0;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x) {
    const double v = b[k] - q[k];
    r[k] = v;
    acc += v * v;
  }
  write_partial(acc, rr.part);
}

void launch_resid_init(const ddeig_problem* P, const double* b, const double* q, double* r,
                       Red& rr, hipStream_t s) {
  rr.np = red_grid(P->g.n);
  hipLaunchKernelGGL(k_resid_init, dim3(rr.np), dim3(kBlock), 0, s, P->g.n, b, q, r, rr);
}

__global__ void k_finish_sum(Red r) {
  const double v = sum_partials(r.part, r.np);
  if (threadIdx.x == 0) *r.val = v;
}

void launch_finish_sum(const Red& r, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kBlock), 0, s, r);
}

__global__ void k_pcg_init(PcgState* st, double rtol, Red rr, double* __restrict__ hist,
                           double rz_floor) {
  pcg_init_body(st, rtol, rr, hist, rz_floor);
}

void launch_pcg_init(const ddeig_problem* P, double rtol, Red rr, hipStream_t s,
                     double rz_floor) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(kBlock), 0, s, P->st, rtol, rr, P->hist, rz_floor);
}

__global__ void k_fill(double* x, long n, double v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    x[i] = v;
}

void launch_fill(double* x, long n, double v, hipStream_t s) {
  const int blocks = (int)std::min<long>((n + kBlock - 1) / kBlock, 4096);
  if (blocks > 0) hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, s, x, n, v);
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    d[i] = s[i];
}

void launch_copy(double* dst, const double* src, long n, hipStream_t s) {
  const int blocks = (int)std::min<long>((n + kBlock - 1) / kBlock, 4096);
  if (blocks > 0) hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kBlock), 0, s, dst, src, n);
}

// dst = src / sqrt(nrm2)  (M-normalisation of a start vector)
__global__ void k_scale_copy(long n, double* __restrict__ dst, const double* __restrict__ src,
                             Red nrm2) {
  const double sc = 1.0 / sqrt(sum_partials(nrm2.part, nrm2.np));
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i] * sc;
}

void launch_scale_copy(long n, double* dst, const double* src, Red nrm2, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(red_grid(n)), dim3(kBlock), 0, s, n, dst, src, nrm2);
}

// Inverse-iteration normalisation (§2): with u = A_sigma^{-1} b, b = M x,
// Mu = M u, scale = sign(1^T M u) / sqrt(u^T M u): x_new = scale u and
// ||x_new - x||_M^2 = (x_new - x)^T (scale Mu - b); x is overwritten by x_new.
__global__ void k_ipm_normalise(long n, const double* __restrict__ u, const double* __restrict__ Mu,
                                double* __restrict__ x, const double* __restrict__ b, Red uMu,
                                Red sumMu, Red dx) {
  const double ssum = sum_partials(sumMu.part, sumMu.np);
  const double uu = sum_partials(uMu.part, uMu.np);
  const double sc = (ssum < 0.0 ? -1.0 : 1.0) / sqrt(uu);
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const double xn = sc * u[i];
    const double d = xn - x[i];
    acc += d * (sc * Mu[i] - b[i]);
    x[i] = xn;
  }
  write_partial(acc, dx.part);
}

void launch_ipm_normalise(long n, const double* u, const double* Mu, double* x, const double* b,
                          Red uMu, Red sumMu, Red& dx, hipStream_t s) {
  dx.np = red_grid(n);
  hipLaunchKernelGGL(k_ipm_normalise, dim3(dx.np), dim3(kBlock), 0, s, n, u, Mu, x, b, uMu,
                     sumMu, dx);
}

__global__ void k_dot(const double* __restrict__ x, const double* __restrict__ y, long n, Red out) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  write_partial(acc, out.part);
}

void launch_dot(const double* x, const double* y, long n, Red& out, hipStream_t s) {
  out.np = red_grid(n);
  hipLaunchKernelGGL(k_dot, dim3(out.np), dim3(kBlock), 0, s, x, y, n, out);
}

__global__ void k_to_float(const double* __restrict__ s, float* __restrict__ d, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    d[i] = (float)s[i];
}

void launch_to_float(const double* src, float* dst, long n, hipStream_t s) {
  const int blocks = (int)std::min<long>((n + kBlock - 1) / kBlock, 4096);
  if (blocks > 0) hipLaunchKernelGGL(k_to_float, dim3(blocks), dim3(kBlock), 0, s, src, dst, n);
}

// ---- SI-preconditioned LOPCG (alg:si-lopcg) ---------------------------------
// Vectors of one outer step, each with its A and B images (B = M):
// x = x_k (B-normalised), w = the preconditioned residual, p = x_k - x_{k-1}.

// B-orthogonalise the search directions against x_k on the vectors themselves
// (their A and B images are then formed from the results, so that the small
// differences near convergence keep their digits): w -= alpha x, and
// p = x_k - x_{k-1} minus its x_k part, which is beta x_k - x_{k-1}
// (alpha = x^T B w, beta = x^T B x_{k-1}; x^T B x = 1).
__global__ void k_lopcg_orth(long n, double alpha, double beta, const double* __restrict__ x,
                             double* __restrict__ w, double* __restrict__ xp) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const double xi = x[i];
    w[i] -= alpha * xi;
    xp[i] = beta * xi - xp[i];
  }
}

void launch_lopcg_orth(long n, double alpha, double beta, const double* x, double* w, double* xp,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_lopcg_orth, dim3(red_grid(n)), dim3(kBlock), 0, s, n, alpha, beta, x, w,
                     xp);
}

// Gram data of S = [s0, s1, s2] = [x, w, p]: out[0..5] = s_i^T A s_j and
// out[6..11] = s_i^T B s_j for (i, j) = (0,0), (0,1), (0,2), (1,1), (1,2),
// (2,2), out[12..14] = 1^T B s_i.  One partial per block and quantity
// (part[q * np + block]); k_lopcg_finish adds them in block order.
__global__ void __launch_bounds__(kBlock) k_lopcg_gram(long n, const double* const* __restrict__ v,
                                                        double* __restrict__ part) {
  const double* S[3] = {v[0], v[1], v[2]};
  const double* AS[3] = {v[3], v[4], v[5]};
  const double* BS[3] = {v[6], v[7], v[8]};
  double acc[kLopcgQ];
#pragma unroll
  for (int q = 0; q < kLopcgQ; ++q) acc[q] = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    double s[3], a[3], b[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s[k] = S[k][i];
      a[k] = AS[k][i];
      b[k] = BS[k][i];
    }
    int q = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = r; c < 3; ++c) {
        acc[q] += s[r] * a[c];
        acc[6 + q] += s[r] * b[c];
        ++q;
      }
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[12 + k] += b[k];
  }
#pragma unroll
  for (int q = 0; q < kLopcgQ; ++q) {
    const double t = block_sum(acc[q]);
    if (threadIdx.x == 0) part[(long)q * gridDim.x + blockIdx.x] = t;
  }
}

// out[q] = sum of the np partials of quantity q, in block order.
__global__ void k_lopcg_finish(const double* __restrict__ part, int np, int nq,
                               double* __restrict__ out) {
  for (int q = 0; q < nq; ++q) {
    const double t = sum_partials(part + (long)q * np, np);
    if (threadIdx.x == 0) out[q] = t;
  }
}

int launch_lopcg_gram(long n, const double* const* dv, double* part, double* out,
                      hipStream_t s) {
  const int np = red_grid(n);
  hipLaunchKernelGGL(k_lopcg_gram, dim3(np), dim3(kBlock), 0, s, n, dv, part);
  hipLaunchKernelGGL(k_lopcg_finish, dim3(1), dim3(kBlock), 0, s, part, np, kLopcgQ, out);
  return np;
}

// x_{k+1} = c0 x + c1 w + c2 p (the Ritz vector, B-normalised by the
// coefficients) and x_{k-1} := x_k.
__global__ void k_lopcg_update(long n, double c0, double c1, double c2, double* __restrict__ x,
                               const double* __restrict__ w, double* __restrict__ p) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const double xo = x[i];
    x[i] = c0 * xo + c1 * w[i] + c2 * p[i];
    p[i] = xo;
  }
}

// r = A x - lambda B x with partials of ||r||^2 (quantity 0 of part).
__global__ void __launch_bounds__(kBlock) k_lopcg_resid(long n, double lambda,
                                                         const double* __restrict__ Ax,
                                                         const double* __restrict__ Bx,
                                                         double* __restrict__ r,
                                                         double* __restrict__ part) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const double v = Ax[i] - lambda * Bx[i];
    r[i] = v;
    acc += v * v;
  }
  write_partial(acc, part);
}

void launch_lopcg_update(long n, double c0, double c1, double c2, double* x, const double* w,
                         double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_lopcg_update, dim3(red_grid(n)), dim3(kBlock), 0, s, n, c0, c1, c2, x, w,
                     p);
}

int launch_lopcg_resid(long n, double lambda, const double* Ax, const double* Bx, double* r,
                       double* part, double* out, hipStream_t s) {
  const int np = red_grid(n);
  hipLaunchKernelGGL(k_lopcg_resid, dim3(np), dim3(kBlock), 0, s, n, lambda, Ax, Bx, r, part);
  hipLaunchKernelGGL(k_lopcg_finish, dim3(1), dim3(kBlock), 0, s, part, np, 1, out);
  return np;
}

}  // namespace ddeig

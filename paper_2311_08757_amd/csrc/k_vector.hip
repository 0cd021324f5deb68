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

__global__ void k_pcg_init(PcgState* st, double rtol, Red rr, double* __restrict__ hist) {
  const double r0n2 = sum_partials(rr.part, rr.np);
  if (threadIdx.x == 0) {
    st->r0n2 = r0n2;
    st->tol2 = rtol * rtol * r0n2;
    st->iters = 0;
    st->rho[0] = st->rho[1] = 0.0;
    st->relres = r0n2 > 0.0 ? 1.0 : 0.0;
    st->done = r0n2 > 0.0 ? 0 : 1;
    if (hist) hist[0] = st->relres;
  }
}

void launch_pcg_init(const ddeig_problem* P, double rtol, Red rr, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(kBlock), 0, s, P->st, rtol, rr, P->hist);
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

}  // namespace ddeig

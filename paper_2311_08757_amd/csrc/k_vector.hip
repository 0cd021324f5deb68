// Vector kernels of preconditioned CG (§3 eq:cg-energy-norm-error-reduction,
// stopping rule of §4.1) and of the shifted inverse iteration with
// B-normalisation (§2).  Scalars stay on the device: each kernel that needs a
// global sum re-reduces the fixed-size partial sums of the kernel before it,
// so no host round trip is needed inside an iteration and sums are
// deterministic.  After convergence or breakdown the state's `done` flag
// turns every later iteration kernel into a no-op, so the host can queue
// several iterations between checks.
#include "k_common.h"

namespace ddeig {

__global__ void k_resid_init(long n, const double* __restrict__ b, const double* __restrict__ q,
                             double* __restrict__ r, double* __restrict__ part) {
  double acc = 0.0;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x) {
    const double v = b[k] - q[k];
    r[k] = v;
    acc += v * v;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_resid_init(const ddeig_problem* P, const double* b, const double* q, double* r,
                       double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_init, dim3(kRedBlocks), dim3(kBlock), 0, s, P->g.n, b, q, r, part);
}

__global__ void k_pcg_init(PcgState* st, double rtol, const double* __restrict__ part,
                           double* __restrict__ hist) {
  const double r0n2 = sum_partials(part);
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

void launch_pcg_init(const ddeig_problem* P, double rtol, const double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(kBlock), 0, s, P->st, rtol, part, P->hist);
}

// p = z, rho_0 = r.z
__global__ void k_pcg_start(long n, PcgState* st, const double* __restrict__ z,
                            double* __restrict__ p, const double* __restrict__ part) {
  const double rho = sum_partials(part);
  if (st->done) return;
  if (!(rho > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 3;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[0] = rho;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x)
    p[k] = z[k];
}

void launch_pcg_start(const ddeig_problem* P, const double* z, double* p, const double* part,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_start, dim3(kRedBlocks), dim3(kBlock), 0, s, P->g.n, P->st, z, p, part);
}

// Iteration k: alpha = rho_{k-1} / (p.q); x += alpha p; r -= alpha q; partials of ||r||^2.
__global__ void k_pcg_update_xr(long n, PcgState* st, int k, double* __restrict__ x,
                                const double* __restrict__ p, const double* __restrict__ q,
                                double* __restrict__ r, const double* __restrict__ part_g,
                                double* __restrict__ part_r) {
  if (st->done) return;
  const double gamma = sum_partials(part_g);
  if (!(gamma > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->done = 2;
      st->iters = k - 1;
    }
    return;
  }
  const double alpha = st->rho[(k - 1) & 1] / gamma;
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double rv = r[i] - alpha * q[i];
    r[i] = rv;
    acc += rv * rv;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part_r[blockIdx.x] = s;
}

void launch_pcg_update_xr(const ddeig_problem* P, double* x, const double* pvec,
                          const double* qvec, double* r, const double* part_g, double* part_r,
                          int k, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_update_xr, dim3(kRedBlocks), dim3(kBlock), 0, s, P->g.n, P->st, k, x,
                     pvec, qvec, r, part_g, part_r);
}

// Convergence test ||r_k|| <= rtol ||r_0|| after the update of iteration k.
__global__ void k_pcg_check(PcgState* st, int k, int maxit, const double* __restrict__ part_r,
                            double* __restrict__ hist, int hist_cap) {
  if (st->done) return;
  const double rn2 = sum_partials(part_r);
  if (threadIdx.x == 0) {
    st->relres = sqrt(rn2 / st->r0n2);
    if (hist && k < hist_cap) hist[k] = st->relres;
    st->iters = k;
    if (rn2 <= st->tol2) st->done = 1;
    else if (k >= maxit) st->done = 4;
  }
}

void launch_pcg_check(const ddeig_problem* P, const double* part_r, int k, int maxit,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(kBlock), 0, s, P->st, k, maxit, part_r, P->hist,
                     P->hist_cap);
}

// beta = rho_k / rho_{k-1}; p = z + beta p.
__global__ void k_pcg_update_p(long n, PcgState* st, int k, const double* __restrict__ z,
                               double* __restrict__ p, const double* __restrict__ part_rz) {
  if (st->done) return;
  const double rho = sum_partials(part_rz);
  if (!(rho > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 3;
    return;
  }
  const double beta = rho / st->rho[(k - 1) & 1];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[k & 1] = rho;
}

void launch_pcg_update_p(const ddeig_problem* P, const double* z, double* pvec,
                         const double* part_rz, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_update_p, dim3(kRedBlocks), dim3(kBlock), 0, s, P->g.n, P->st, k, z,
                     pvec, part_rz);
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

// dst = src / sqrt(sum(part))  (mode 0: M-normalisation of a start vector)
__global__ void k_scale_copy(long n, double* __restrict__ dst, const double* __restrict__ src,
                             const double* __restrict__ part) {
  const double nrm2 = sum_partials(part);
  const double sc = 1.0 / sqrt(nrm2);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i] * sc;
}

void launch_scale_copy(long n, double* dst, const double* src, const double* part,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(kRedBlocks), dim3(kBlock), 0, s, n, dst, src, part);
}

// Inverse-iteration normalisation (§2): with u = A_sigma^{-1} b, b = M x,
// Mu = M u, scale = sign(1^T M u) / sqrt(u^T M u): x_new = scale u and the
// partials of ||x_new - x||_M^2 = (x_new - x)^T (scale Mu - b); x is
// overwritten by x_new.
__global__ void k_ipm_normalise(long n, const double* __restrict__ u, const double* __restrict__ Mu,
                                double* __restrict__ x, const double* __restrict__ b,
                                const double* __restrict__ part_uMu,
                                const double* __restrict__ part_sum,
                                double* __restrict__ part_dx) {
  const double uMu = sum_partials(part_uMu);
  const double ssum = sum_partials(part_sum);
  const double sc = (ssum < 0.0 ? -1.0 : 1.0) / sqrt(uMu);
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const double xn = sc * u[i];
    const double d = xn - x[i];
    acc += d * (sc * Mu[i] - b[i]);
    x[i] = xn;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part_dx[blockIdx.x] = s;
}

void launch_ipm_normalise(long n, const double* u, const double* Mu, double* x, const double* b,
                          const double* part_uMu, const double* part_sum, double* part_dx,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_normalise, dim3(kRedBlocks), dim3(kBlock), 0, s, n, u, Mu, x, b,
                     part_uMu, part_sum, part_dx);
}

__global__ void k_sum_partials(const double* __restrict__ part, double* __restrict__ out) {
  const double v = sum_partials(part);
  if (threadIdx.x == 0) *out = v;
}

void launch_sum_partials(const double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, part, out);
}

__global__ void k_dot(const double* __restrict__ x, const double* __restrict__ y, long n,
                      double* __restrict__ part) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_dot(const double* x, const double* y, long n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(kBlock), 0, s, x, y, n, part);
}

}  // namespace ddeig

namespace ddeig {

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

// Vector kernels of the stationary restricted additive Schwarz iteration
// (eq:stationary-ras, eq:two-level-stationary-ras-mult-cc) and of GMRES with
// right preconditioning (§3: the unsymmetric M_RAS,2 is used inside GMRES).
//
// As in CG, scalars stay on the device and every global sum adds per-block
// partials in a fixed order, so the iterations are deterministic and the host
// only checks the state every few steps.  Every kernel here is a no-op once the
// state's `done` flag is set.
//
// GMRES keeps its Arnoldi basis V (restart + 1 vectors) and the preconditioned
// vectors Z_j = M^{-1} v_j (restart vectors) in one workspace, each vector at
// a stride of ldv doubles.  One step j: z_j = M^{-1} v_j, w = A_sigma z_j
// written into v_{j+1}, classical Gram-Schmidt applied twice against
// v_0..v_j (each pass: block partials of the dots, their fixed-order sums,
// then the update), ||w|| folded into the second update, and one single-block
// kernel that completes column j of the Hessenberg matrix, applies the
// previous Givens rotations and the new one, and decides whether to stop.
// The solution update x += Z y uses the stored Z (flexible form), so a
// preconditioner that rounds its input (bf16 local solves) still gives the
// Arnoldi relation A Z_m = V_{m+1} H_m exactly as computed.
#include "k_common.h"

namespace ddeig {

// x += z (a correction of the stationary iteration).
__global__ void k_sr_update(long n, const PcgState* __restrict__ st, const double* __restrict__ z,
                            double* __restrict__ x) {
  if (st->done) return;
  for (long k = blockIdx.x * (long)kBlock + threadIdx.x; k < n; k += (long)gridDim.x * kBlock)
    x[k] += z[k];
}

void launch_sr_update(const ddeig_problem* P, const double* z, double* x, hipStream_t s) {
  const int blocks = (int)std::max<long>(1, std::min<long>((P->g.n + kBlock - 1) / kBlock, 4096));
  hipLaunchKernelGGL(k_sr_update, dim3(blocks), dim3(kBlock), 0, s, P->g.n, P->st, z, x);
}

// Stopping test after step k of the stationary iteration: ||r_k|| <= rtol ||r_0||.
__global__ void k_sr_check(PcgState* __restrict__ st, Red rr, int k, int maxit,
                           double* __restrict__ hist, int hist_cap) {
  if (st->done) return;
  const double rn2 = sum_partials(rr.part, rr.np);
  if (threadIdx.x == 0) {
    st->relres = sqrt(rn2 / st->r0n2);
    st->iters = k;
    if (hist && k < hist_cap) hist[k] = st->relres;
    if (rn2 <= st->tol2) st->done = 1;
    else if (k >= maxit) st->done = 4;
    else if (!(rn2 == rn2) || rn2 > 1e300) st->done = 2;  // diverged to inf / NaN
  }
}

void launch_sr_check(const ddeig_problem* P, const Red& rr, int k, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(k_sr_check, dim3(1), dim3(kBlock), 0, s, P->st, rr, k, maxit, P->hist,
                     P->hist_cap);
}

// ---------------------------------------------------------------------------
// GMRES

// Nodes per thread of the basis kernels: a block owns kBlock * kGmE consecutive
// nodes, so the partial-sum grid is n / (kBlock * kGmE) rounded up.
constexpr int kGmE = 4;

int gm_blocks(long n) { return (int)std::max<long>(1, (n + kBlock * kGmE - 1) / (kBlock * kGmE)); }

// part[v * nblk + b] = block b's partial of v_v . w, v = 0..nv-1.
__global__ void __launch_bounds__(kBlock) k_gm_dots(long n, int nv, const double* __restrict__ V,
                                                    long ldv, const double* __restrict__ w,
                                                    const PcgState* __restrict__ st,
                                                    double* __restrict__ part) {
  if (st->done) return;
  const long base = (long)blockIdx.x * kBlock * kGmE + threadIdx.x;
  double wr[kGmE];
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    wr[e] = k < n ? w[k] : 0.0;
  }
  for (int v = 0; v < nv; ++v) {
    const double* vp = V + (long)v * ldv;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < kGmE; ++e) {
      const long k = base + (long)kBlock * e;
      if (k < n) acc += vp[k] * wr[e];
    }
    write_partial_at(acc, part + (long)v * gridDim.x, blockIdx.x);
  }
}

// out[v] = sum over the nblk partials of vector v, in block order (one block per v).
__global__ void __launch_bounds__(kBlock) k_gm_sum(const double* __restrict__ part, int nblk,
                                                   const PcgState* __restrict__ st,
                                                   double* __restrict__ out) {
  if (st->done) return;
  const double v = sum_partials(part + (long)blockIdx.x * nblk, nblk);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// w -= sum_v h[v] v_v (v in order); with nrm, the partials of ||w||^2 go to nrm.
__global__ void __launch_bounds__(kBlock) k_gm_axpy(long n, int nv, const double* __restrict__ V,
                                                    long ldv, const double* __restrict__ h,
                                                    double* __restrict__ w,
                                                    const PcgState* __restrict__ st,
                                                    double* __restrict__ nrm) {
  if (st->done) return;
  const long base = (long)blockIdx.x * kBlock * kGmE + threadIdx.x;
  double wr[kGmE];
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    wr[e] = k < n ? w[k] : 0.0;
  }
  for (int v = 0; v < nv; ++v) {
    const double c = h[v];
    const double* vp = V + (long)v * ldv;
#pragma unroll
    for (int e = 0; e < kGmE; ++e) {
      const long k = base + (long)kBlock * e;
      if (k < n) wr[e] -= c * vp[k];
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    if (k < n) {
      w[k] = wr[e];
      acc += wr[e] * wr[e];
    }
  }
  if (nrm) write_partial_at(acc, nrm, blockIdx.x);
}

// Column j of the Hessenberg matrix (column-major, ldh = restart + 1 rows):
// H[0..j, j] = h1 + h2, H[j+1, j] = ||w||, then the rotations of the columns
// before and the new rotation that zeroes H[j+1, j]; g (the rotated
// right-hand side beta e_1) gives the residual norm |g[j+1]| of step k (the
// k-th of the whole solve).  done: 1 converged (including ||w|| = 0), 2
// breakdown (a zero column), 4 maxit, 6 end of the restart cycle.
// gm[0] receives 1 / ||w|| for the normalisation of v_{j+1}.
__global__ void k_gm_finish(int j, int k, int maxit, int restart, const double* __restrict__ nrm,
                            int nblk, const double* __restrict__ h1, const double* __restrict__ h2,
                            double* __restrict__ H, double* __restrict__ cs,
                            double* __restrict__ sn, double* __restrict__ g,
                            double* __restrict__ gm, PcgState* __restrict__ st,
                            double* __restrict__ hist, int hist_cap) {
  if (st->done) return;
  const double nw2 = sum_partials(nrm, nblk);
  if (threadIdx.x != 0) return;
  double* Hc = H + (long)j * (restart + 1);
  for (int i = 0; i <= j; ++i) Hc[i] = h1[i] + h2[i];
  const double hn = sqrt(nw2);
  Hc[j + 1] = hn;
  gm[0] = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * Hc[i] + sn[i] * Hc[i + 1];
    Hc[i + 1] = -sn[i] * Hc[i] + cs[i] * Hc[i + 1];
    Hc[i] = t;
  }
  const double den = hypot(Hc[j], Hc[j + 1]);
  st->iters = k;
  if (!(den > 0.0)) {
    st->done = 2;
    return;
  }
  cs[j] = Hc[j] / den;
  sn[j] = Hc[j + 1] / den;
  Hc[j] = den;
  Hc[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  const double res2 = g[j + 1] * g[j + 1];
  st->relres = sqrt(res2 / st->r0n2);
  if (hist && k < hist_cap) hist[k] = st->relres;
  if (res2 <= st->tol2 || hn == 0.0) st->done = 1;
  else if (k >= maxit) st->done = 4;
  else if (j + 1 >= restart) st->done = 6;
}

// v = w * gm[0] in place (the normalised next basis vector).
__global__ void k_gm_scale(long n, double* __restrict__ w, const double* __restrict__ gm,
                           const PcgState* __restrict__ st) {
  if (st->done) return;
  const double c = gm[0];
  for (long k = blockIdx.x * (long)kBlock + threadIdx.x; k < n; k += (long)gridDim.x * kBlock)
    w[k] *= c;
}

// Start of a cycle from the residual r (partials rr): beta = ||r||, g = beta e_1,
// v_0 = r / beta.  done = 1 when beta^2 <= tol2 (or beta = 0), else 0.
__global__ void k_gm_start(Red rr, double* __restrict__ g, double* __restrict__ gm,
                           PcgState* __restrict__ st) {
  const double b2 = sum_partials(rr.part, rr.np);
  if (threadIdx.x == 0) {
    const double beta = sqrt(b2);
    g[0] = beta;
    gm[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    st->done = (b2 <= st->tol2 || beta == 0.0) ? 1 : 0;
  }
}

__global__ void k_gm_scale_copy(long n, const double* __restrict__ r, double* __restrict__ v,
                                const double* __restrict__ gm, const PcgState* __restrict__ st) {
  if (st->done) return;
  const double c = gm[0];
  for (long k = blockIdx.x * (long)kBlock + threadIdx.x; k < n; k += (long)gridDim.x * kBlock)
    v[k] = r[k] * c;
}

// x += sum_v y[v] Z_v (v in order).
__global__ void __launch_bounds__(kBlock) k_gm_update(long n, int nv, const double* __restrict__ Z,
                                                      long ldv, const double* __restrict__ y,
                                                      double* __restrict__ x) {
  const long base = (long)blockIdx.x * kBlock * kGmE + threadIdx.x;
  double xr[kGmE];
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    xr[e] = k < n ? x[k] : 0.0;
  }
  for (int v = 0; v < nv; ++v) {
    const double c = y[v];
    const double* zp = Z + (long)v * ldv;
#pragma unroll
    for (int e = 0; e < kGmE; ++e) {
      const long k = base + (long)kBlock * e;
      if (k < n) xr[e] += c * zp[k];
    }
  }
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    if (k < n) x[k] = xr[e];
  }
}

static int elem_grid(long n) {
  return (int)std::max<long>(1, std::min<long>((n + kBlock - 1) / kBlock, 4096));
}

void launch_gm_dots(const ddeig_problem* P, int nv, const double* V, long ldv, const double* w,
                    double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_dots, dim3(gm_blocks(P->g.n)), dim3(kBlock), 0, s, P->g.n, nv, V, ldv, w,
                     P->st, part);
}

void launch_gm_sum(const ddeig_problem* P, int nv, const double* part, double* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_gm_sum, dim3(nv), dim3(kBlock), 0, s, part, gm_blocks(P->g.n), P->st, out);
}

void launch_gm_axpy(const ddeig_problem* P, int nv, const double* V, long ldv, const double* h,
                    double* w, double* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_axpy, dim3(gm_blocks(P->g.n)), dim3(kBlock), 0, s, P->g.n, nv, V, ldv, h,
                     w, P->st, nrm);
}

void launch_gm_finish(const ddeig_problem* P, int j, int k, int maxit, int restart,
                      const double* nrm, const double* h1, const double* h2, double* H, double* cs,
                      double* sn, double* g, double* gm, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_finish, dim3(1), dim3(kBlock), 0, s, j, k, maxit, restart, nrm,
                     gm_blocks(P->g.n), h1, h2, H, cs, sn, g, gm, P->st, P->hist, P->hist_cap);
}

void launch_gm_scale(const ddeig_problem* P, double* w, const double* gm, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_scale, dim3(elem_grid(P->g.n)), dim3(kBlock), 0, s, P->g.n, w, gm,
                     P->st);
}

void launch_gm_start(const ddeig_problem* P, const Red& rr, const double* r, double* v0, double* g,
                     double* gm, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_start, dim3(1), dim3(kBlock), 0, s, rr, g, gm, P->st);
  hipLaunchKernelGGL(k_gm_scale_copy, dim3(elem_grid(P->g.n)), dim3(kBlock), 0, s, P->g.n, r, v0,
                     gm, P->st);
}

void launch_gm_update(const ddeig_problem* P, int nv, const double* Z, long ldv, const double* y,
                      double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_update, dim3(gm_blocks(P->g.n)), dim3(kBlock), 0, s, P->g.n, nv, Z, ldv,
                     y, x);
}

}  // namespace ddeig

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
// vectors z_j = M^{-1} u_j (restart vectors) in one workspace, each vector at a
// stride of ldv doubles.  The Arnoldi process is classical Gram-Schmidt with
// the second (re-)orthogonalisation pass delayed by one step (DCGS2, Bielich,
// Langou, Thomas, Swirydowicz, Yamazaki and Boman, 2022): step j applies the
// preconditioner and the operator to u_j, the vector left by step j-1 after
// one projection (scaled, not yet normalised), then
//   one dot sweep over v_0..v_{j-1} gives V^T u_j, V^T w, u.u, u.w, w.w;
//   a single-thread kernel finishes column j-1 of the Hessenberg matrix with
//   the second projection of u_j, applies the Givens rotations and the
//   stopping test, and forms column j's first-pass entries;
//   one update sweep writes v_j (u_j reorthogonalised and normalised) and
//   u_{j+1} (w projected once).
// That is two sweeps over the basis per step instead of four for classical
// Gram-Schmidt applied twice.  Since w_j = A z_j is expressed exactly in the
// orthonormal V, the relation A Z = V H holds for the vectors actually used
// (flexible GMRES), so x = x0 + Z y is right also when the local solves round
// their input (bf16).
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
// Basis vectors per batched block reduction of the dot kernel.
constexpr int kGmVB = 8;

int gm_blocks(long n) { return (int)std::max<long>(1, (n + kBlock * kGmE - 1) / (kBlock * kGmE)); }

// Reduces VB values per thread over the workgroup (fixed order: shuffle tree in
// each wave64, then the waves in order); thread b < VB receives total b.
template <int VB>
__device__ inline double block_sum_batch(double (&v)[VB]) {
  __shared__ double sh[VB][kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < VB; ++b)
    for (int off = 32; off > 0; off >>= 1) v[b] += __shfl_down(v[b], off, 64);
  __syncthreads();  // earlier readers of sh are done
  if (lane == 0)
#pragma unroll
    for (int b = 0; b < VB; ++b) sh[b][w] = v[b];
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < VB)
    for (int i = 0; i < kBlock / 64; ++i) t += sh[threadIdx.x][i];
  return t;
}

// The dot products of step j of the delayed Gram-Schmidt Arnoldi process
// (one sweep over v_0..v_{j-1}): with u = u_j (basis slot j) and w = A z_j,
// rows of part (nblk partials each):
//   i < j: v_i.u;  j: u.u;  and when w is given  j+1+i: v_i.w (i < j),
//   2j+1: u.w,  2j+2: w.w.
// Block (c, q) takes node chunk c (kBlock * kGmE nodes) and basis vectors
// q kGmVG .. q kGmVG + kGmVG - 1 (group 0 also the three scalars), so a step
// has chunks x groups workgroups.  Vectors are zero beyond n up to ldv (the
// work space is cleared when allocated and only entries below n are written),
// so the loads need no bounds test.
constexpr int kGmVG = 16;

__global__ void __launch_bounds__(kBlock) k_gm_dots(int j, const double* __restrict__ V, long ldv,
                                                    const double* __restrict__ w,
                                                    const PcgState* __restrict__ st,
                                                    double* __restrict__ part) {
  if (st->done) return;
  const long nb = gridDim.x;
  const long base = (long)blockIdx.x * kBlock * kGmE + threadIdx.x;
  const double* u = V + (long)j * ldv;
  double ur[kGmE], wr[kGmE];
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    ur[e] = u[k];
    wr[e] = w != nullptr ? w[k] : 0.0;
  }
  const int vend = min(j, (int)(blockIdx.y + 1) * kGmVG);
  for (int v0 = blockIdx.y * kGmVG; v0 < vend; v0 += kGmVB) {
    double acc[2 * kGmVB];
#pragma unroll
    for (int b = 0; b < kGmVB; ++b) {
      acc[b] = acc[kGmVB + b] = 0.0;
      if (v0 + b < vend) {
        const double* vp = V + (long)(v0 + b) * ldv;
#pragma unroll
        for (int e = 0; e < kGmE; ++e) {
          const double x = vp[base + (long)kBlock * e];
          acc[b] += x * ur[e];
          acc[kGmVB + b] += x * wr[e];
        }
      }
    }
    const double t = block_sum_batch<2 * kGmVB>(acc);
    const int b = threadIdx.x % kGmVB;
    if (threadIdx.x < 2 * kGmVB && v0 + b < vend) {
      if (threadIdx.x < kGmVB) part[(long)(v0 + b) * nb + blockIdx.x] = t;
      else if (w != nullptr) part[(long)(j + 1 + v0 + b) * nb + blockIdx.x] = t;
    }
  }
  if (blockIdx.y != 0) return;
  double sc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    sc[0] += ur[e] * ur[e];
    sc[1] += ur[e] * wr[e];
    sc[2] += wr[e] * wr[e];
  }
  const double t = block_sum_batch<3>(sc);
  if (threadIdx.x == 0) part[(long)j * nb + blockIdx.x] = t;
  if (w != nullptr && threadIdx.x >= 1 && threadIdx.x < 3)
    part[(long)(2 * j + threadIdx.x) * nb + blockIdx.x] = t;
}

// out[row] = the sum of the nblk partials of the row, in block order (one block per row).
__global__ void __launch_bounds__(kBlock) k_gm_sum(const double* __restrict__ part, int nblk,
                                                   const PcgState* __restrict__ st,
                                                   double* __restrict__ out) {
  if (st->done) return;
  const double v = sum_partials(part + (long)blockIdx.x * nblk, nblk);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// Scalars of step j, from the sums d of k_gm_dots (one wave64: the vectors of
// the step are staged in LDS and reduced across the wave; only the rotation
// chain is serial):
// 1. the second projection of u_j: u_j = V_j s + alpha v_j, s = d[0..j-1],
//    alpha^2 = u.u - ||s||^2 (u_j was projected once already, so little cancels);
// 2. column j-1 of H gets its second-pass terms: the first-pass entries stored at
//    step j-1 plus s / c_{j-1}, and H[j, j-1] = alpha / c_{j-1} (u_j was w_{j-1}'s
//    remainder scaled by c_{j-1}); then the rotations and the stopping test of
//    iteration k;
// 3. with w (a full step, not done): the projections of w on v_0..v_j,
//    p_i = d[j+1+i] and h = v_j.w = (u.w - s.p) / alpha, stored as column j's
//    first-pass entries, and the scale c_j = 1 / ||w - V p - h v_j|| from
//    Pythagoras (any positive scale keeps the recurrence exact: it is carried
//    into step j+1).
// gm[0] = 1 / alpha, gm[1] = h, gm[2] = c_j for the update.  Step 0 takes
// v_0 = u_0 (alpha = 1).  The wave's sums use a fixed shuffle order.
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(64) k_gm_decide(int j, int k, int maxit, int restart, int has_w,
                                                  const double* __restrict__ d,
                                                  double* __restrict__ H, double* __restrict__ cs,
                                                  double* __restrict__ sn, double* __restrict__ g,
                                                  double* __restrict__ cv, double* __restrict__ gm,
                                                  PcgState* __restrict__ st,
                                                  double* __restrict__ hist, int hist_cap) {
  __shared__ double hc[kGmMaxRestart + 1], lc[kGmMaxRestart], ls[kGmMaxRestart];
  __shared__ int done;
  const int t = threadIdx.x;
  if (t == 0) done = st->done;
  __syncthreads();
  if (done) return;
  const long ldh = restart + 1;
  double alpha = 1.0;
  if (j > 0) {
    double ss = 0.0;
    for (int i = t; i < j; i += 64) ss += d[i] * d[i];
    ss = wave_sum(ss);
    const double a2 = d[j] - ss;
    alpha = a2 > 0.0 ? sqrt(a2) : 0.0;
    double* Hp = H + (long)(j - 1) * ldh;
    const double c = cv[j - 1];
    for (int i = t; i < j; i += 64) hc[i] = Hp[i] + d[i] / c;
    for (int i = t; i < j - 1; i += 64) {
      lc[i] = cs[i];
      ls[i] = sn[i];
    }
    __syncthreads();
    if (t == 0) {
      // rotations of the earlier columns, then the new one, on column j-1
      const int col = j - 1;
      const double nu = alpha / c;
      double carry = hc[0];
      for (int i = 0; i < col; ++i) {
        const double a = carry, b = hc[i + 1];
        hc[i] = lc[i] * a + ls[i] * b;
        carry = -ls[i] * a + lc[i] * b;
      }
      hc[col] = carry;
      hc[col + 1] = nu;
      const double den = hypot(hc[col], hc[col + 1]);
      st->iters = k;
      if (!(den > 0.0)) {
        st->done = 2;
      } else {
        const double cc = hc[col] / den, sc = hc[col + 1] / den;
        cs[col] = cc;
        sn[col] = sc;
        hc[col] = den;
        hc[col + 1] = 0.0;
        const double gc = g[col];
        g[col + 1] = -sc * gc;
        g[col] = cc * gc;
        const double res2 = g[col + 1] * g[col + 1];
        st->relres = sqrt(res2 / st->r0n2);
        if (hist && k < hist_cap) hist[k] = st->relres;
        if (res2 <= st->tol2 || nu == 0.0) st->done = 1;
        else if (k >= maxit) st->done = 4;
        else if (col + 1 >= restart) st->done = 6;
      }
      done = st->done;
    }
    __syncthreads();
    for (int i = t; i <= j; i += 64) Hp[i] = hc[i];
    if (done) return;
  }
  if (!has_w) {  // a closing step always ends the cycle
    if (t == 0) st->done = 6;
    return;
  }
  double sp = 0.0, pp = 0.0;
  for (int i = t; i < j; i += 64) {
    const double pi = d[j + 1 + i];
    sp += d[i] * pi;
    pp += pi * pi;
  }
  sp = wave_sum(sp);
  pp = wave_sum(pp);
  const double uw = d[2 * j + 1], ww = d[2 * j + 2];
  const double h = (uw - sp) / alpha;
  double* Hc = H + (long)j * ldh;
  for (int i = t; i < j; i += 64) Hc[i] = d[j + 1 + i];
  if (t == 0) {
    Hc[j] = h;
    const double nu2 = ww - pp - h * h;
    const double c = nu2 > 1e-30 * ww ? 1.0 / sqrt(nu2) : (ww > 0.0 ? 1.0 / sqrt(ww) : 1.0);
    cv[j] = c;
    gm[0] = 1.0 / alpha;
    gm[1] = h;
    gm[2] = c;
  }
}

// The update sweep of step j over v_0..v_{j-1}: v_j = (u_j - V s) / alpha in
// place of u_j (basis slot j), and u_{j+1} = (w - V p - h v_j) c_j into slot
// j+1, with s = d[0..j-1], p = d[j+1..2j] (sums in index order).
__global__ void __launch_bounds__(kBlock) k_gm_update_basis(long n, int j, double* __restrict__ V,
                                                            long ldv, const double* __restrict__ w,
                                                            const double* __restrict__ d,
                                                            const double* __restrict__ gm,
                                                            const PcgState* __restrict__ st) {
  if (st->done) return;
  const double ia = gm[0], h = gm[1], c = gm[2];
  double* u = V + (long)j * ldv;
  double* un = V + (long)(j + 1) * ldv;
  const long base = (long)blockIdx.x * kBlock * kGmE + threadIdx.x;
  double su[kGmE], sw[kGmE];
#pragma unroll
  for (int e = 0; e < kGmE; ++e) su[e] = sw[e] = 0.0;
#pragma unroll 4
  for (int i = 0; i < j; ++i) {
    const double a = d[i], b = d[j + 1 + i];
    const double* vp = V + (long)i * ldv;
#pragma unroll
    for (int e = 0; e < kGmE; ++e) {
      const double x = vp[base + (long)kBlock * e];
      su[e] += a * x;
      sw[e] += b * x;
    }
  }
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const long k = base + (long)kBlock * e;
    if (k < n) {
      const double vj = (u[k] - su[e]) * ia;
      u[k] = vj;
      un[k] = (w[k] - sw[e] - h * vj) * c;
    }
  }
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
#pragma unroll 8
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

void launch_gm_dots(const ddeig_problem* P, int j, const double* V, long ldv, const double* w,
                    double* part, hipStream_t s) {
  const int groups = std::max(1, (j + kGmVG - 1) / kGmVG);
  hipLaunchKernelGGL(k_gm_dots, dim3(gm_blocks(P->g.n), groups), dim3(kBlock), 0, s, j, V, ldv, w,
                     P->st, part);
}

// Vector stride of the GMRES work space: n rounded up to whole node chunks of
// the basis kernels (their loads run unguarded to the stride).
long gm_stride(long n) {
  const long chunk = (long)kBlock * kGmE;
  return (n + chunk - 1) / chunk * chunk;
}

void launch_gm_sum(const ddeig_problem* P, int rows, const double* part, double* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_gm_sum, dim3(rows), dim3(kBlock), 0, s, part, gm_blocks(P->g.n), P->st, out);
}

void launch_gm_decide(const ddeig_problem* P, int j, int k, int maxit, int restart, int has_w,
                      const double* d, double* H, double* cs, double* sn, double* g, double* cv,
                      double* gm, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_decide, dim3(1), dim3(64), 0, s, j, k, maxit, restart, has_w, d, H, cs,
                     sn, g, cv, gm, P->st, P->hist, P->hist_cap);
}

void launch_gm_update_basis(const ddeig_problem* P, int j, double* V, long ldv, const double* w,
                            const double* d, const double* gm, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_update_basis, dim3(gm_blocks(P->g.n)), dim3(kBlock), 0, s, P->g.n, j, V,
                     ldv, w, d, gm, P->st);
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

// Device helpers shared by the kernels: deterministic block reductions,
// stencil tap decoding, the periodic potential and node/table indexing.
#pragma once
#include "ddeig_internal.h"

namespace ddeig {

// FP64 -> bf16 correctly rounded (to nearest, ties to even) in one step; the
// residuals and inverses of the bf16 local solves are rounded with it.
__device__ inline __bf16 to_bf16(double x) { return (__bf16)x; }


// Sum over a workgroup of NT threads; every thread receives the total.  The
// order of additions is fixed (shuffle tree inside each wave64, then the
// waves in order), so repeated runs give identical bits.
template <int NT>
__device__ inline double block_sum_n(double v) {
  __shared__ double sh_red[NT / 64 + 1];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh_red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t += sh_red[i];
    sh_red[NT / 64] = t;
  }
  __syncthreads();
  return sh_red[NT / 64];
}

__device__ inline double block_sum(double v) { return block_sum_n<kBlock>(v); }

// One partial sum per block (see Red); bid is the block's index among the
// producers of the sum (its blockIdx.x, or its index within one instance of a
// grouped launch).
template <int NT = kBlock>
__device__ inline void write_partial_at(double v, double* part, int bid) {
  const double b = block_sum_n<NT>(v);
  if (threadIdx.x == 0) part[bid] = b;
}

template <int NT = kBlock>
__device__ inline void write_partial(double v, double* part) {
  write_partial_at<NT>(v, part, blockIdx.x);
}

// The sum of the np partials of a producing kernel, added in block order by
// a workgroup of NT threads.
template <int NT = kBlock>
__device__ inline double sum_partials(const double* part, int np) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += NT) v += part[i];
  return block_sum_n<NT>(v);
}

// Start of PCG (stopping rule of §4.1): ||r_0||^2 from the partials of rr,
// the tolerance, an empty direction history; CG is finished at once when
// r_0 = 0.  Run by one workgroup of kBlock threads.
__device__ inline void pcg_init_body(PcgState* st, double rtol, const Red& rr,
                                     double* __restrict__ hist, double rz_floor) {
  const double r0n2 = sum_partials(rr.part, rr.np);
  if (threadIdx.x == 0) {
    st->rz_floor = rz_floor;
    st->r0n2 = r0n2;
    st->tol2 = rtol * rtol * r0n2;
    st->iters = 0;
    st->rho[0] = st->rho[1] = 0.0;
    st->relres = r0n2 > 0.0 ? 1.0 : 0.0;
    st->done = r0n2 > 0.0 ? 0 : 1;
    if (hist) hist[0] = st->relres;
  }
}

// Offsets of tap t; with ntaps = 9 (2-D) there is no third dim and d2 = 0.
__device__ inline void tap_offsets(int t, int ntaps, int& d0, int& d1, int& d2) {
  d0 = t % 3 - 1;
  d1 = (t / 3) % 3 - 1;
  d2 = ntaps == 9 ? 0 : t / 9 - 1;
}

// Table node of the unknown with 0-based indices (i0, i1, i2): x dims use the
// cell-local node index (i + 1) mod n_e, y dims the unknown index itself.
__device__ inline long table_node(const Geo& g, int i0, int i1, int i2) {
  int j0 = g.isx[0] ? (i0 + 1) % g.ne : i0;
  int j1 = g.isx[1] ? (i1 + 1) % g.ne : i1;
  int j2 = (g.D == 3 && g.isx[2]) ? (i2 + 1) % g.ne : i2;
  return (long)j0 + (long)g.P[0] * ((long)j1 + (long)g.P[1] * j2);
}

// V at a point z (x cell-local), as documented in ddeig_potential.
__host__ __device__ inline double eval_V(const VSpec& v, const double* z) {
  const double two_pi = 6.283185307179586476925286766559;
  const double pi = 3.1415926535897932384626433832795;
  double out = 0.0;
  switch (v.kind) {
    case DDEIG_V_CONST:
      out = v.c0;
      break;
    case DDEIG_V_SEP_FOURIER: {
      double F = 0.0;
      for (int t = 0; t < v.nterms; ++t) F += v.a[t] * cos(two_pi * v.k[t] * z[0] + v.phi[t]);
      double G = 1.0;
      for (int j = 0; j < v.q; ++j) G *= sin(pi * z[v.p + j] / v.ell);
      out = F * (1.0 + v.cy * G);
      break;
    }
    case DDEIG_V_FOURIER2: {
      for (int t = 0; t < v.nterms; ++t)
        out += v.a[t] * cos(two_pi * (v.k[t] * z[0] + v.m[t] * z[1]) + v.phi[t]);
      break;
    }
    case DDEIG_V_SIN4: {
      out = v.c0;
      for (int i = 0; i < v.p; ++i) {
        double s = sin(pi * z[i]);
        out *= s * s * s * s;
      }
      for (int j = 0; j < v.q; ++j) {
        double s = sin(pi * z[v.p + j] / v.ell);
        out *= s * s * s * s;
      }
      break;
    }
    case DDEIG_V_SEP_SUM: {
      out = v.c0;
      for (int t = 0; t < v.nterms; ++t) out += v.a[t] * sin(two_pi * v.k[t] * z[v.m[t]]);
      for (int j = 0; j < v.q; ++j) out += v.g[j] * z[v.p + j];
      break;
    }
    default:
      out = 0.0;
  }
  return out;
}

__device__ inline FastDiv make_fastdiv_dev(unsigned d) {
  FastDiv f{d, 0u, 0u};
  unsigned s = 0;
  while ((1ull << s) < d) ++s;
  f.shift = s;
  f.mul = (unsigned)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}

__device__ inline unsigned fdiv(unsigned n, const FastDiv& f) {
  return (unsigned)(((unsigned long long)__umulhi(n, f.mul) + n) >> f.shift);
}

__device__ inline void unflatten(const Geo& g, long k, int& i0, int& i1, int& i2) {
  i0 = (int)(k % g.N[0]);
  long r = k / g.N[0];
  i1 = (int)(r % g.N[1]);
  i2 = (int)(r / g.N[1]);
}

}  // namespace ddeig

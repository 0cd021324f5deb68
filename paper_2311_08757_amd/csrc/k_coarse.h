// Device bodies of the coarse correction of the two-level preconditioner
// (eq:two-level-preconditioners, def:algebraic-perfact-coarse-space), shared by
// the coarse kernels and by the launches that carry them as extra workgroups
// (the dense GEMM carries R_0 r, the clipped-class correction A_0^{-1} c).
#pragma once
#include "k_common.h"

namespace ddeig {

// c_sub = phi_class . R_sub r  (R_0 r of def:algebraic-perfact-coarse-space):
// one workgroup per subdomain.  Thread t takes the box elements t + kBlock q
// (natural order; the grid line from a multiply-high division), 8 at a time
// with all 16 loads issued before the products; the products are added in q
// order, then the threads in a fixed order.
__device__ __forceinline__ void coarse_rhs_body(const Geo& g, const PcgState* __restrict__ st,
                                                const double* __restrict__ r,
                                                const TypeDev* __restrict__ types,
                                                const SubDev* __restrict__ subs,
                                                double* __restrict__ crhs, int bid) {
  if (st != nullptr && st->done) return;
  const SubDev sd = subs[bid];
  const TypeDev td = types[sd.type];
  const int m0 = td.m[0], m1 = td.m[1];
  const int mtot = m0 * m1 * td.m[2];
  constexpr int U = 8;
  double acc = 0.0;
  for (int e0 = threadIdx.x; e0 < mtot; e0 += U * kBlock) {
    double ph[U], rv[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = e0 + q * kBlock;
      ph[q] = rv[q] = 0.0;
      if (e < mtot) {
        const int line = (int)fdiv((unsigned)e, td.fm0);
        const int u0 = e - line * m0;
        const int u2 = line / m1, u1 = line - u2 * m1;
        ph[q] = td.phi[e];
        rv[q] = r[(sd.o[0] + u0) + (long)g.N[0] * ((sd.o[1] + u1) + (long)g.N[1] * (sd.o[2] + u2))];
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) acc += ph[q] * rv[q];
  }
  const double sum = block_sum(acc);
  if (threadIdx.x == 0) crhs[bid] = sum;
}

// y0 = A0^{-1} c with the dense symmetric inverse: one wave64 per row, lanes
// stride the row (coalesced), fixed-order shuffle reduction.
__device__ __forceinline__ void coarse_solve_body(int N, const PcgState* __restrict__ st,
                                                  const double* __restrict__ A0inv,
                                                  const double* __restrict__ c,
                                                  double* __restrict__ y, int bid) {
  if (st != nullptr && st->done) return;
  const int lane = threadIdx.x & 63;
  const int row = bid * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= N) return;
  double acc = 0.0;
  for (int j = lane; j < N; j += 64) acc += A0inv[(long)row * N + j] * c[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[row] = acc;
}

}  // namespace ddeig

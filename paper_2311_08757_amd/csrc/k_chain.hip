// Block-tridiagonal ("chain") factorisation and solves of box operators.
//
// The local matrices A_sigma,i = R_i A_sigma R_i^T of §3
// (eq:twoLevelASMPreconditioner) and the cell operator of
// eq:weak-form-cell-problem are the stencil operator restricted to a box of
// unknowns.  Ordered slice by slice along the last (fixed, Dirichlet) grid
// direction they are block tridiagonal: diagonal blocks D_i (couplings inside
// slice i, with the periodic wrap of the cell problem inside the slice) and
// sub-diagonal blocks E_i (slice i to slice i-1).  Block elimination gives
//   S_0 = D_0,  S_i = D_i - E_i S_{i-1}^{-1} E_i^T,  W_i = S_i^{-1},
// and a solve is
//   forward   t_i = W_i (b_i - E_i t_{i-1}),
//   backward  x_{n-1} = t_{n-1},  x_i = t_i - W_i E_{i+1}^T x_{i+1}.
// E_i and D_i are never stored: they are read from the period-cell table.
// W_i is stored dense (b x b); since it is symmetric, W_i[s][r] is read with
// r running over the threads, which coalesces.
#include "k_common.h"

namespace ddeig {

// In-slice neighbour of box-local u (slice coordinates a < D-1) along tap d.
__device__ inline bool slice_nbr(const Box& bx, int D, const int* u, const int* d, int& rn) {
  int idx = 0, stride = 1;
  for (int a = 0; a < D - 1; ++a) {
    int w = u[a] + d[a];
    if (bx.per[a]) w = (w + bx.m[a]) % bx.m[a];
    else if (w < 0 || w >= bx.m[a]) return false;
    idx += w * stride;
    stride *= bx.m[a];
  }
  rn = idx;
  return true;
}

__device__ inline void slice_coords(const Box& bx, int D, int r, int* u) {
  u[0] = 0; u[1] = 0; u[2] = 0;
  for (int a = 0; a < D - 1; ++a) {
    u[a] = r % bx.m[a];
    r /= bx.m[a];
  }
}

__device__ inline long box_tnode(const Geo& g, const Box& bx, const int* u) {
  return table_node(g, bx.o[0] + u[0], bx.o[1] + u[1], bx.o[2] + u[2]);
}

// S = D_i - E_i Wprev E_i^T for slice i (Wprev = nullptr for i = 0), row-major b x b.
__global__ void k_schur_build(Geo g, Box bx, int i, const double* __restrict__ T,
                              const double* __restrict__ Wprev, double* __restrict__ S) {
  const int b = bx.b, D = g.D, last = D - 1;
  const long bb = (long)b * b;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < bb;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / b), s = (int)(idx % b);
    int ur[3], us[3];
    slice_coords(bx, D, r, ur);
    slice_coords(bx, D, s, us);
    ur[last] = i;
    us[last] = i;
    const long tr = box_tnode(g, bx, ur);
    double v = 0.0;
    for (int t = 0; t < g.ntaps; ++t) {
      int d[3];
      tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
      if (d[last] != 0) continue;
      int rn;
      if (slice_nbr(bx, D, ur, d, rn) && rn == s) v += T[t * g.tsize + tr];
    }
    if (Wprev != nullptr) {
      const long ts = box_tnode(g, bx, us);
      double corr = 0.0;
      for (int t1 = 0; t1 < g.ntaps; ++t1) {
        int d1[3];
        tap_offsets(t1, g.ntaps, d1[0], d1[1], d1[2]);
        if (d1[last] != -1) continue;
        int n1;
        if (!slice_nbr(bx, D, ur, d1, n1)) continue;
        const double e1 = T[t1 * g.tsize + tr];
        double inner = 0.0;
        for (int t2 = 0; t2 < g.ntaps; ++t2) {
          int d2[3];
          tap_offsets(t2, g.ntaps, d2[0], d2[1], d2[2]);
          if (d2[last] != -1) continue;
          int n2;
          if (!slice_nbr(bx, D, us, d2, n2)) continue;
          inner += T[t2 * g.tsize + ts] * Wprev[(long)n1 * b + n2];
        }
        corr += e1 * inner;
      }
      v -= corr;
    }
    S[idx] = v;
  }
}

// Gauss-Jordan inversion in place, one launch per pivot.  rowk/colk hold row
// and column k of the matrix before step k; the launch also records row and
// column k+1 after step k into rown/coln for the next pivot.
__global__ void k_gj_step(double* __restrict__ A, int b, int k, const double* __restrict__ rowk,
                          const double* __restrict__ colk, double* __restrict__ rown,
                          double* __restrict__ coln, int* __restrict__ flag) {
  const double piv = rowk[k];
  if (!(piv > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    return;
  }
  const double ipiv = 1.0 / piv;
  const long bb = (long)b * b;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < bb;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / b), j = (int)(idx % b);
    double v;
    if (i == k) {
      v = (j == k) ? ipiv : rowk[j] * ipiv;
    } else {
      const double f = colk[i];
      v = (j == k) ? -f * ipiv : A[idx] - f * (rowk[j] * ipiv);
    }
    A[idx] = v;
    if (i == k + 1) rown[j] = v;
    if (j == k + 1) coln[i] = v;
  }
}

__global__ void k_gj_init(const double* __restrict__ A, int b, double* __restrict__ row0,
                          double* __restrict__ col0) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < b; j += gridDim.x * blockDim.x) {
    row0[j] = A[j];
    col0[j] = A[(long)j * b];
  }
}

void launch_gj_invert(ddeig_problem* P, double* A, int b, hipStream_t s) {
  const long st = P->gj_stride;
  double* bufs[2][2] = {{P->gjbuf, P->gjbuf + st}, {P->gjbuf + 2 * st, P->gjbuf + 3 * st}};
  hipLaunchKernelGGL(k_gj_init, dim3((b + kBlock - 1) / kBlock), dim3(kBlock), 0, s, A, b,
                     bufs[0][0], bufs[0][1]);
  const long bb = (long)b * b;
  const int blocks = (int)std::min<long>((bb + kBlock - 1) / kBlock, 4096);
  for (int k = 0; k < b; ++k) {
    double** cur = bufs[k & 1];
    double** nxt = bufs[(k + 1) & 1];
    hipLaunchKernelGGL(k_gj_step, dim3(blocks), dim3(kBlock), 0, s, A, b, k, cur[0], cur[1],
                       nxt[0], nxt[1], P->flag);
  }
}

void chain_factor(ddeig_problem* P, const Box& bx, const double* tab, double* W, hipStream_t s) {
  const long bb = (long)bx.b * bx.b;
  const int blocks = (int)std::min<long>((bb + kBlock - 1) / kBlock, 4096);
  for (int i = 0; i < bx.nch; ++i) {
    double* Wi = W + (long)i * bb;
    const double* Wp = i > 0 ? W + (long)(i - 1) * bb : nullptr;
    hipLaunchKernelGGL(k_schur_build, dim3(blocks), dim3(kBlock), 0, s, P->g, bx, i, tab, Wp, Wi);
    launch_gj_invert(P, Wi, bx.b, s);
  }
}

// One workgroup solves one right-hand side v (nch * b values, slice-major,
// overwritten by the solution).  sh holds 2 b doubles of LDS.
template <typename WT>
__device__ void chain_solve_block(const Geo& g, const Box& bx, const double* __restrict__ T,
                                  const WT* __restrict__ W, double* __restrict__ v, double* sh) {
  const int b = bx.b, nch = bx.nch, D = g.D, last = D - 1;
  double* gb = sh;
  double* tb = sh + b;
  const long bb = (long)b * b;
  // forward sweep
  for (int i = 0; i < nch; ++i) {
    for (int r = threadIdx.x; r < b; r += blockDim.x) {
      double val = v[(long)i * b + r];
      if (i > 0) {
        int u[3];
        slice_coords(bx, D, r, u);
        u[last] = i;
        const long tn = box_tnode(g, bx, u);
        for (int t = 0; t < g.ntaps; ++t) {
          int d[3];
          tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
          if (d[last] != -1) continue;
          int rn;
          if (slice_nbr(bx, D, u, d, rn)) val -= T[t * g.tsize + tn] * tb[rn];
        }
      }
      gb[r] = val;
    }
    __syncthreads();
    const WT* Wi = W + (long)i * bb;
    for (int r = threadIdx.x; r < b; r += blockDim.x) {
      double acc = 0.0;
      for (int s2 = 0; s2 < b; ++s2) acc += (double)Wi[(long)s2 * b + r] * gb[s2];
      v[(long)i * b + r] = acc;
      tb[r] = acc;
    }
    __syncthreads();
  }
  // backward sweep; tb holds x_{i+1}
  for (int i = nch - 2; i >= 0; --i) {
    for (int r = threadIdx.x; r < b; r += blockDim.x) {
      int u[3];
      slice_coords(bx, D, r, u);
      u[last] = i;
      const long tn = box_tnode(g, bx, u);
      double val = 0.0;
      for (int t = 0; t < g.ntaps; ++t) {
        int d[3];
        tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
        if (d[last] != 1) continue;
        int rn;
        if (slice_nbr(bx, D, u, d, rn)) val += T[t * g.tsize + tn] * tb[rn];
      }
      gb[r] = val;
    }
    __syncthreads();
    const WT* Wi = W + (long)i * bb;
    for (int r = threadIdx.x; r < b; r += blockDim.x) {
      double acc = 0.0;
      for (int s2 = 0; s2 < b; ++s2) acc += (double)Wi[(long)s2 * b + r] * gb[s2];
      const double x = v[(long)i * b + r] - acc;
      v[(long)i * b + r] = x;
      tb[r] = x;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_chain_solve_box(Geo g, Box bx,
                                                            const double* __restrict__ T,
                                                            const double* __restrict__ W,
                                                            double* __restrict__ v) {
  extern __shared__ double sh[];
  chain_solve_block<double>(g, bx, T, W, v + (long)blockIdx.x * bx.nch * bx.b, sh);
}

void launch_chain_solve_box(const ddeig_problem* P, const Box& bx, const double* tab,
                            const double* W, double* v, int nrhs, hipStream_t s) {
  const size_t lds = 2 * (size_t)bx.b * sizeof(double);
  hipLaunchKernelGGL(k_chain_solve_box, dim3(nrhs), dim3(kBlock), lds, s, P->g, bx, tab, W, v);
}

// All local subdomain solves of the level-1 preconditioner in one launch:
// workgroup = subdomain, solved with its class's shared factor.
template <typename WT>
__global__ void __launch_bounds__(kBlock) k_local_solves(Geo g, const double* __restrict__ T,
                                                         const TypeDev* __restrict__ types,
                                                         const SubDev* __restrict__ subs,
                                                         const PcgState* __restrict__ st) {
  extern __shared__ double sh[];
  if (st != nullptr && st->done) return;
  const SubDev sd = subs[blockIdx.x];
  const TypeDev td = types[sd.type];
  Box bx;
  for (int a = 0; a < 3; ++a) {
    bx.o[a] = sd.o[a];
    bx.m[a] = td.m[a];
    bx.per[a] = 0;
  }
  bx.b = td.b;
  bx.nch = td.nch;
  const WT* W;
  if constexpr (sizeof(WT) == 4) W = reinterpret_cast<const WT*>(td.W32);
  else W = reinterpret_cast<const WT*>(td.W);
  chain_solve_block<WT>(g, bx, T, W, td.batch + (long)sd.slot * td.nch * td.b, sh);
}

// ---- batched chain solves
//
// All members of a class share the factors W_i, so a sweep step is the same
// for every member: forward t_i = W_i (b_i - E_i t_{i-1}), backward
// x_i = t_i - W_i E_{i+1}^T x_{i+1}.  A step is three launches:
//   k_chain_rhs: the right-hand sides g of every member (the coupling taps
//     from the table), thread per row, into a buffer [member][row];
//   k_chain_mm: workgroup (row tile of 64 rows, K chunk, member group of up
//     to 64 members of one class) stages its K chunk of g in LDS and
//     multiplies it by rows [r0, r0 + 64) of W_i restricted to the chunk
//     (lane = row, reading W_i by columns since it is symmetric, which
//     coalesces; wave = 16 members); the partial products go to a buffer
//     [K chunk][member][row];
//   k_chain_fin: adds the K-chunk partials of each (member, row) in chunk
//     order and writes t_i (forward) or x_i = t_i - (sum) (backward).
// W_i is read once per member group and step, and a step has row tiles x
// K chunks x groups workgroups.  Arithmetic in WT (FP64, or FP32 for
// local_prec 1) with the right-hand sides formed in FP64.  3-D boxes only
// (chain along the last dim, slices of the first two).
template <typename WT>
struct ChainCfg {
  static constexpr int RT = 64;                         // rows per workgroup
  static constexpr int KC = 64;                         // K chunk (16 or 32 KB of LDS)
  static constexpr int MG = 64;                         // members per group
};

// The right-hand sides g of step i for every member of a job, once per step:
// row r of member m into G[(mg0 + m) * bmax + r] (thread per row).
template <typename WT, bool FWD>
__global__ void __launch_bounds__(kBlock) k_chain_rhs(Geo g, const double* __restrict__ T,
                                                      const TypeDev* __restrict__ types,
                                                      const ChainJob* __restrict__ jobs, int i,
                                                      int bmax, WT* __restrict__ G,
                                                      const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  const ChainJob jb = jobs[blockIdx.y];
  const TypeDev td = types[jb.type];
  const int b = td.b, nch = td.nch;
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= b || (int)blockIdx.z >= jb.nm) return;
  const long mstride = (long)nch * b;
  const int m0 = td.m[0], m1 = td.m[1];
  const bool couple = FWD ? i > 0 : true;
  const int j = FWD ? i - 1 : i + 1;
  const double* nb = FWD ? td.tbatch : td.batch;
  // the 9 taps with d2 = -1 (forward) or +1 (backward), in tap order
  const int u1 = r / m0, u0 = r - u1 * m0;
  const long tn = table_node(g, td.o[0] + u0, td.o[1] + u1, td.o[2] + i);
  const int d2 = FWD ? -1 : 1;
  double c[9];
  int nbr[9];
#pragma unroll
  for (int t9 = 0; t9 < 9; ++t9) {
    const int d0 = t9 % 3 - 1, d1 = t9 / 3 - 1;
    const int w0 = u0 + d0, w1 = u1 + d1;
    const bool in = couple && w0 >= 0 && w0 < m0 && w1 >= 0 && w1 < m1;
    c[t9] = in ? T[(t9 + 9 * (d2 + 1)) * g.tsize + tn] : 0.0;
    nbr[t9] = in ? w0 + m0 * w1 : r;
  }
  const int m = blockIdx.z;  // the member (grid z covers a job's members)
  const long base = (long)(jb.m0 + m) * mstride;
  double acc = FWD ? td.batch[base + (long)i * b + r] : 0.0;
  if (couple) {
    const double* nbs = nb + base + (long)j * b;
#pragma unroll
    for (int t9 = 0; t9 < 9; ++t9) acc += (FWD ? -c[t9] : c[t9]) * nbs[nbr[t9]];
  }
  G[(long)(jb.mg0 + m) * bmax + r] = (WT)acc;
}

template <typename WT>
__global__ void __launch_bounds__(kBlock) k_chain_mm(const TypeDev* __restrict__ types,
                                                     const ChainJob* __restrict__ jobs, int i,
                                                     int mtot, int bmax,
                                                     const WT* __restrict__ G,
                                                     WT* __restrict__ part,
                                                     const PcgState* __restrict__ st) {
  using C = ChainCfg<WT>;
  __shared__ __attribute__((aligned(16))) WT gs[C::KC][C::MG];
  if (st != nullptr && st->done) return;
  const ChainJob jb = jobs[blockIdx.z];
  const TypeDev td = types[jb.type];
  const int b = td.b;
  const int r0 = blockIdx.x * C::RT, k0 = blockIdx.y * C::KC;
  if (r0 >= b || k0 >= b) return;
  const int kn = min(C::KC, b - k0);
  // the chunk of the right-hand sides (row fastest: coalesced reads)
  for (int idx = threadIdx.x; idx < kn * C::MG; idx += kBlock) {
    const int m = idx / kn, k = idx - m * kn;
    gs[k][m] = m < jb.nm ? G[(long)(jb.mg0 + m) * bmax + k0 + k] : (WT)0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = r0 + lane;
  constexpr int MW = C::MG / (kBlock / 64);  // members per wave
  WT acc[MW];
#pragma unroll
  for (int q = 0; q < MW; ++q) acc[q] = (WT)0;
  if (r < b && wv * MW < jb.nm) {
    const WT* Wi = (sizeof(WT) == 4 ? reinterpret_cast<const WT*>(td.W32)
                                    : reinterpret_cast<const WT*>(td.W)) +
                   (long)i * b * b + (long)k0 * b + r;
    constexpr int KB = 32;  // loads of W_i in flight per lane
    for (int kk = 0; kk < kn; kk += KB) {
      WT w[KB];
#pragma unroll
      for (int q = 0; q < KB; ++q) w[q] = kk + q < kn ? Wi[(long)(kk + q) * b] : (WT)0;
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        // (past the chunk w[q] = 0 multiplies the chunk's last, written, row);
        // the wave's MW values of the row are read 16 bytes at a time (every
        // lane reads the same address: a broadcast)
        typedef __attribute__((__vector_size__(16))) WT wvec;
        constexpr int VW = 16 / sizeof(WT);
        const wvec* gk = reinterpret_cast<const wvec*>(&gs[min(kk + q, kn - 1)][wv * MW]);
#pragma unroll
        for (int v4 = 0; v4 < MW / VW; ++v4) {
          const wvec gv = gk[v4];
#pragma unroll
          for (int e = 0; e < VW; ++e) acc[v4 * VW + e] += w[q] * gv[e];
        }
      }
    }
  }
  if (r >= b) return;
#pragma unroll
  for (int mm = 0; mm < MW; ++mm) {
    const int m = wv * MW + mm;
    if (m < jb.nm) part[((long)blockIdx.y * mtot + jb.mg0 + m) * bmax + r] = acc[mm];
  }
}

// t_i = sum of the K-chunk partials (forward), x_i = t_i - sum (backward),
// x_{n-1} = t_{n-1} (copy, the first backward step).
template <typename WT, bool FWD>
__global__ void __launch_bounds__(kBlock) k_chain_fin(const TypeDev* __restrict__ types,
                                                      const ChainJob* __restrict__ jobs, int i,
                                                      int mtot, int bmax,
                                                      const WT* __restrict__ part, int copy,
                                                      const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  const ChainJob jb = jobs[blockIdx.y];
  const TypeDev td = types[jb.type];
  const int b = td.b;
  const int r = blockIdx.x * kBlock + threadIdx.x;
  const int m = blockIdx.z;  // the member (grid z covers a job's members)
  if (r >= b || m >= jb.nm) return;
  const int nkc = (b + ChainCfg<WT>::KC - 1) / ChainCfg<WT>::KC;
  const long mstride = (long)td.nch * b;
  const long at = (long)(jb.m0 + m) * mstride + (long)i * b + r;
  if (copy) {
    td.batch[at] = td.tbatch[at];
    return;
  }
  double v = 0.0;
  for (int kc = 0; kc < nkc; ++kc) v += (double)part[((long)kc * mtot + jb.mg0 + m) * bmax + r];
  if (FWD) td.tbatch[at] = v;
  else td.batch[at] = td.tbatch[at] - v;
}

// Members per group of the batched chain solves and the partial buffer size.
int chain_group_members() { return ChainCfg<double>::MG; }

size_t chain_part_bytes(int bmax, int mtot, int fp32) {
  // the K-chunk partials, then the right-hand sides
  const int kc = fp32 ? ChainCfg<float>::KC : ChainCfg<double>::KC;
  return (size_t)((bmax + kc - 1) / kc + 1) * mtot * bmax * (fp32 ? sizeof(float) : sizeof(double));
}

template <typename WT>
static void chain_sweeps(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  using C = ChainCfg<WT>;
  const int nch = P->types[0].box.nch;
  const int bmax = P->chain_bmax, mtot = P->chain_mtot;
  const int nkc = (bmax + C::KC - 1) / C::KC;
  WT* part = reinterpret_cast<WT*>(P->chain_part);
  WT* G = part + (long)nkc * mtot * bmax;
  const dim3 gmm((bmax + C::RT - 1) / C::RT, nkc, P->nchainjobs);
  const dim3 gnode((bmax + kBlock - 1) / kBlock, P->nchainjobs, C::MG);
  for (int i = 0; i < nch; ++i) {
    hipLaunchKernelGGL((k_chain_rhs<WT, true>), gnode, dim3(kBlock), 0, s, P->g, P->tabAs,
                       P->dTypes, P->dChainJobs, i, bmax, G, st);
    hipLaunchKernelGGL((k_chain_mm<WT>), gmm, dim3(kBlock), 0, s, P->dTypes, P->dChainJobs, i,
                       mtot, bmax, G, part, st);
    hipLaunchKernelGGL((k_chain_fin<WT, true>), gnode, dim3(kBlock), 0, s, P->dTypes,
                       P->dChainJobs, i, mtot, bmax, part, 0, st);
  }
  hipLaunchKernelGGL((k_chain_fin<WT, false>), gnode, dim3(kBlock), 0, s, P->dTypes,
                     P->dChainJobs, nch - 1, mtot, bmax, part, 1, st);
  for (int i = nch - 2; i >= 0; --i) {
    hipLaunchKernelGGL((k_chain_rhs<WT, false>), gnode, dim3(kBlock), 0, s, P->g, P->tabAs,
                       P->dTypes, P->dChainJobs, i, bmax, G, st);
    hipLaunchKernelGGL((k_chain_mm<WT>), gmm, dim3(kBlock), 0, s, P->dTypes, P->dChainJobs, i,
                       mtot, bmax, G, part, st);
    hipLaunchKernelGGL((k_chain_fin<WT, false>), gnode, dim3(kBlock), 0, s, P->dTypes,
                       P->dChainJobs, i, mtot, bmax, part, 0, st);
  }
}

void launch_chain_batched(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  if (P->opt.local_prec == 1) chain_sweeps<float>(P, st, s);
  else chain_sweeps<double>(P, st, s);
}

bool local_solves_fast_ok(const ddeig_problem* P);
void launch_local_solves_fast(const ddeig_problem* P, const PcgState* st, hipStream_t s);

void launch_local_solves(const ddeig_problem* P, const PcgState* st, hipStream_t s,
                         const double* coarse_r) {
  if (P->opt.local_prec >= 2) {
    // one batch of all subdomains: MFMA tiles, or the streaming kernel for a
    // handful of rows (one of the two has no work); coarse_r (nullable): the
    // GEMM launch also forms R_0 coarse_r
    launch_dense_gemm(P, st, s, coarse_r);
    launch_dense_gemv(P, st, s);
    return;
  }
  if (local_solves_fast_ok(P)) {
    launch_local_solves_fast(P, st, s);
    return;
  }
  if (P->nchainjobs > 0) {
    if (P->chain_mfma) launch_chain_mfma(P, st, s);
    else launch_chain_batched(P, st, s);
    return;
  }
  const size_t lds = 2 * (size_t)P->maxb * sizeof(double);
  if (P->opt.local_prec == 1)
    hipLaunchKernelGGL(k_local_solves<float>, dim3(P->nsub), dim3(kBlock), lds, s, P->g,
                       P->tabAs, P->dTypes, P->dSubs, st);
  else
    hipLaunchKernelGGL(k_local_solves<double>, dim3(P->nsub), dim3(kBlock), lds, s, P->g,
                       P->tabAs, P->dTypes, P->dSubs, st);
}

}  // namespace ddeig

namespace ddeig {

// Local solves of the 2-D decompositions (slices along x of at most kFastB
// unknowns, chain along y).  W_i is staged in LDS with double buffering;
// while step i computes from LDS, every thread already holds its share of
// W_{i+1} (W_{i-1} in the backward sweep), the next slice of the right-hand
// side and the next coupling coefficients in registers.  Each row's dot
// product is split over np = floor(256 / b) thread groups and the parts are
// added in a fixed order.  In 2-D the couplings to the neighbouring slice are
// the taps (d0, d1) = (-1..1, -1) (forward) and (-1..1, +1) (backward), i.e.
// table taps 0..2 and 6..8, with in-slice neighbours r-1, r, r+1.
constexpr int kFastB = 72;
constexpr int kFastRegs = (kFastB * kFastB + kBlock - 1) / kBlock;
template <typename WT>
__device__ inline double dot_part(const WT* __restrict__ wc, const double* __restrict__ gv, int b,
                                  int r, int s0, int s1) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int s = s0;
  for (; s + 3 < s1; s += 4) {
    a0 += (double)wc[s * b + r] * gv[s];
    a1 += (double)wc[(s + 1) * b + r] * gv[s + 1];
    a2 += (double)wc[(s + 2) * b + r] * gv[s + 2];
    a3 += (double)wc[(s + 3) * b + r] * gv[s + 3];
  }
  for (; s < s1; ++s) a0 += (double)wc[s * b + r] * gv[s];
  return (a0 + a1) + (a2 + a3);
}
template <typename WT>
__global__ void __launch_bounds__(kBlock) k_local_solves_2d(Geo g, const double* __restrict__ T,
                                                            const TypeDev* __restrict__ types,
                                                            const SubDev* __restrict__ subs,
                                                            const PcgState* __restrict__ st) {
  __shared__ WT wbuf[2][kFastB * kFastB];
  __shared__ double gb[kFastB];
  __shared__ double tb[kFastB];
  __shared__ double red[kBlock];
  if (st != nullptr && st->done) return;
  const SubDev sd = subs[blockIdx.x];
  const TypeDev td = types[sd.type];
  const int b = td.b, nch = td.nch;
  const int bb = b * b;
  const int tid = threadIdx.x;
  const int np = kBlock / b;  // thread groups per row
  const int chunk = (b + np - 1) / np;
  const int part = tid / b, rr = tid - part * b;
  const bool dot_thread = part < np;
  const int s0 = min(b, part * chunk), s1 = min(b, s0 + chunk);
  const WT* __restrict__ W;
  if constexpr (sizeof(WT) == 4) W = reinterpret_cast<const WT*>(td.W32);
  else W = reinterpret_cast<const WT*>(td.W);
  double* __restrict__ v = td.batch + (long)sd.slot * nch * b;
  const bool row = tid < b;
  const int jx = row ? (sd.o[0] + tid + 1) % g.ne : 0;
  const bool has_l = tid > 0, has_r = tid + 1 < b;
  WT pre[kFastRegs];
  for (int j = tid; j < bb; j += kBlock) wbuf[0][j] = W[j];
  double vnext = row ? v[tid] : 0.0;
  double cn0 = 0.0, cn1 = 0.0, cn2 = 0.0;
  __syncthreads();
  // forward sweep: t_i = W_i (b_i - E_i t_{i-1})
  for (int i = 0; i < nch; ++i) {
    const double vi = vnext, c0 = cn0, c1 = cn1, c2 = cn2;
    if (i + 1 < nch) {
      const WT* Wn = W + (long)(i + 1) * bb;
#pragma unroll
      for (int j = 0; j < kFastRegs; ++j) {
        const int idx = tid + j * kBlock;
        if (idx < bb) pre[j] = Wn[idx];
      }
      if (row) {
        vnext = v[(long)(i + 1) * b + tid];
        const long tn = jx + (long)g.P[0] * (sd.o[1] + i + 1);
        cn0 = T[0 * g.tsize + tn];
        cn1 = T[1 * g.tsize + tn];
        cn2 = T[2 * g.tsize + tn];
      }
    }
    if (row) {
      double val = vi;
      if (i > 0) {
        if (has_l) val -= c0 * tb[tid - 1];
        val -= c1 * tb[tid];
        if (has_r) val -= c2 * tb[tid + 1];
      }
      gb[tid] = val;
    }
    __syncthreads();
    if (dot_thread) red[tid] = dot_part(wbuf[i & 1], gb, b, rr, s0, s1);
    __syncthreads();
    if (row) {
      double acc = red[tid];
      for (int pp = 1; pp < np; ++pp) acc += red[pp * b + tid];
      v[(long)i * b + tid] = acc;
      tb[tid] = acc;
    }
    if (i + 1 < nch) {
#pragma unroll
      for (int j = 0; j < kFastRegs; ++j) {
        const int idx = tid + j * kBlock;
        if (idx < bb) wbuf[(i + 1) & 1][idx] = pre[j];
      }
    }
    __syncthreads();
  }
  // backward sweep: x_i = t_i - W_i E_{i+1}^T x_{i+1}; W_{nch-2} is still in wbuf[nch & 1]
  if (nch >= 2 && row) {
    const long tn = jx + (long)g.P[0] * (sd.o[1] + nch - 2);
    cn0 = T[6 * g.tsize + tn];
    cn1 = T[7 * g.tsize + tn];
    cn2 = T[8 * g.tsize + tn];
    vnext = v[(long)(nch - 2) * b + tid];
  }
  for (int i = nch - 2; i >= 0; --i) {
    const double vi = vnext, c0 = cn0, c1 = cn1, c2 = cn2;
    if (i >= 1) {
      const WT* Wn = W + (long)(i - 1) * bb;
#pragma unroll
      for (int j = 0; j < kFastRegs; ++j) {
        const int idx = tid + j * kBlock;
        if (idx < bb) pre[j] = Wn[idx];
      }
      if (row) {
        vnext = v[(long)(i - 1) * b + tid];
        const long tn = jx + (long)g.P[0] * (sd.o[1] + i - 1);
        cn0 = T[6 * g.tsize + tn];
        cn1 = T[7 * g.tsize + tn];
        cn2 = T[8 * g.tsize + tn];
      }
    }
    if (row) {
      double val = c1 * tb[tid];
      if (has_l) val += c0 * tb[tid - 1];
      if (has_r) val += c2 * tb[tid + 1];
      gb[tid] = val;
    }
    __syncthreads();
    if (dot_thread) red[tid] = dot_part(wbuf[i & 1], gb, b, rr, s0, s1);
    __syncthreads();
    if (row) {
      double acc = red[tid];
      for (int pp = 1; pp < np; ++pp) acc += red[pp * b + tid];
      const double x = vi - acc;
      v[(long)i * b + tid] = x;
      tb[tid] = x;
    }
    if (i >= 1) {
#pragma unroll
      for (int j = 0; j < kFastRegs; ++j) {
        const int idx = tid + j * kBlock;
        if (idx < bb) wbuf[(i - 1) & 1][idx] = pre[j];
      }
    }
    __syncthreads();
  }
}

bool local_solves_fast_ok(const ddeig_problem* P) { return P->maxb <= kFastB && P->g.D == 2; }

void launch_local_solves_fast(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  if (P->opt.local_prec == 1)
    hipLaunchKernelGGL(k_local_solves_2d<float>, dim3(P->nsub), dim3(kBlock), 0, s, P->g,
                       P->tabAs, P->dTypes, P->dSubs, st);
  else
    hipLaunchKernelGGL(k_local_solves_2d<double>, dim3(P->nsub), dim3(kBlock), 0, s, P->g,
                       P->tabAs, P->dTypes, P->dSubs, st);
}

}  // namespace ddeig

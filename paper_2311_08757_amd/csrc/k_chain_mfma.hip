// Batched block-chain local solves of 3-D boxes with FP32 factors on MFMA.
//
// The local matrices A_sigma,i of §3 (eq:twoLevelASMPreconditioner) are block
// tridiagonal along the last (fixed) direction; their block elimination gives
// W_i = S_i^{-1} per slice (k_chain.hip), and a solve is
//   forward   t_i = W_i (b_i - E_i t_{i-1}),
//   backward  x_{n-1} = t_{n-1},  x_i = t_i - W_i E_{i+1}^T x_{i+1}.
// All members of a class share W_i, so each sweep step is one product of W_i
// (b x b, FP32) with the right-hand sides of all members of the class.  A step
// is two launches:
//   k_cm_rhs: finishes the previous step (t_{i-1} in the forward sweep,
//     x_{i+1} in the backward one, as the fixed-order sum of the previous
//     product's K-chunk partials, less t_{i+1} in the backward sweep), stores
//     it for the workgroup's own rows, and forms this step's right-hand sides
//     g from it with the coupling taps of the period-cell table.  The previous
//     step's values are gathered into LDS for the workgroup's rows and a halo
//     of one slice line on each side, which covers every coupling tap.
//   k_cm_mm: the product W_i g on v_mfma_f32_32x32x2f32: workgroup = 128 rows
//     x 64 members x one K chunk of 72, four waves of 32 rows x 64 members (two
//     32 x 32 tiles sharing the W_i fragment; the second is skipped when the
//     job has at most 32 members), so W_i is read once per class; W_i rows
//     of the chunk and g are staged through LDS with coalesced loads (W_i is
//     symmetric, so its rows are the columns of the A operand), the partial
//     tile goes out through LDS so that every wave writes whole rows.
// One more launch after the backward sweep finishes x_0.  The right-hand sides
// are formed and the partials summed in FP64; W_i, g and the products are FP32
// (FP32 accumulation on the matrix cores).
#include "k_common.h"

namespace ddeig {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kCmRows = 128;    // output rows per product workgroup
constexpr int kCmKc = 72;       // K chunk per product workgroup (a slice of 35 x 31 in 16 chunks)
constexpr int kCmMembers = 64;  // members per job: two 32-wide MFMA tiles per wave
constexpr int kCmRb = 256;      // rows per right-hand-side workgroup
constexpr int kCmHalo = 256;    // largest halo (one slice line + 1) of the rhs kernel
constexpr int kCmMaxKc = 32;    // largest number of K chunks (slices of at most 2304 nodes)
constexpr int kCmLdw = kCmRows + 4;  // LDS row of the staged W_i chunk (bank offset per row)

// FP64 factors (rows of b values) -> FP32 rows of ldw values, zero padded.
__global__ void k_pad_float(const double* __restrict__ src, float* __restrict__ dst, long rows,
                            int b, int ldw) {
  const long tot = rows * ldw;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const long r = idx / ldw;
    const int c = (int)(idx - r * ldw);
    dst[idx] = c < b ? (float)src[r * b + c] : 0.0f;
  }
}

void launch_pad_float(const double* src, float* dst, long rows, int b, int ldw, hipStream_t s) {
  const long tot = rows * ldw;
  const int blocks = (int)std::min<long>((tot + kBlock - 1) / kBlock, 8192);
  if (blocks > 0)
    hipLaunchKernelGGL(k_pad_float, dim3(blocks), dim3(kBlock), 0, s, src, dst, rows, b, ldw);
}

int chain_mfma_members() { return kCmMembers; }

bool chain_mfma_ok(int b, int m0) {
  return m0 + 1 <= kCmHalo && b >= 1 && b <= kCmMaxKc * kCmKc;
}

// Previous step's value of row r of member (slot) m: the sum of the nkc K-chunk
// partials of its class (b / kCmKc rounded up, at most MAXK) in chunk order,
// subtracted from t (backward, sub != nullptr).  Every load is issued before
// the first add (clamped addresses, masked values), so their latencies overlap;
// MAXK (16 or 32, the batch's largest chunk count rounded up) bounds the loads.
template <int MAXK>
__device__ inline double cm_prev(const float* __restrict__ part, int nkc, int mtot, int bmax,
                                 int slot, int r, const double* sub) {
  float v[MAXK];
#pragma unroll
  for (int kc = 0; kc < MAXK; ++kc)
    v[kc] = part[((long)min(kc, nkc - 1) * mtot + slot) * bmax + r];
  double acc = 0.0;
#pragma unroll
  for (int kc = 0; kc < MAXK; ++kc)
    if (kc < nkc) acc += (double)v[kc];
  return sub != nullptr ? *sub - acc : acc;
}

// Right-hand sides of sweep step i.  Grid: (row blocks, jobs, members of a job).
// FWD: t_{i-1} from the partials (i > 0) into tbatch, g = b_i - E_i t_{i-1}.
// BWD: x_{i+1} = (i + 1 == nch - 1 ? 0 : t_{i+1}) - ... : the partials of the
// product of step i + 1 are W_{i+1} E_{i+2}^T x_{i+2}, or t_{n-1} itself after
// the last forward step; x_{i+1} into batch, g = E_{i+1}^T x_{i+1}.
template <bool FWD, int MAXK>
__global__ void __launch_bounds__(kBlock) k_cm_rhs(Geo g, const double* __restrict__ T,
                                                   const TypeDev* __restrict__ types,
                                                   const ChainJob* __restrict__ jobs, int i,
                                                   int mtot, int bmax,
                                                   const float* __restrict__ part,
                                                   float* __restrict__ G,
                                                   const PcgState* __restrict__ st) {
  __shared__ double prev[kCmRb + 2 * kCmHalo];
  if (st != nullptr && st->done) return;
  const ChainJob jb = jobs[blockIdx.y];
  const int m = blockIdx.z;
  if (m >= jb.nm) return;
  const TypeDev td = types[jb.type];
  const int b = td.b, nch = td.nch;
  const int nkc = (b + kCmKc - 1) / kCmKc;
  const int R0 = blockIdx.x * kCmRb;
  if (R0 >= b) return;
  const int m0 = td.m[0], m1 = td.m[1];
  const int H = m0 + 1;
  const int slot = jb.mg0 + m;
  const long base = (long)(jb.m0 + m) * nch * b;
  const bool couple = FWD ? i > 0 : true;
  if (couple) {
    // the previous step's values on rows [R0 - H, R0 + kCmRb + H) of the slice
    const int j = FWD ? i - 1 : i + 1;
    const int lo = max(R0 - H, 0), hi = min(R0 + kCmRb + H, b);
    for (int r = lo + threadIdx.x; r < hi; r += kBlock) {
      double v;
      if (FWD || j == nch - 1) {
        v = cm_prev<MAXK>(part, nkc, mtot, bmax, slot, r, nullptr);
      } else {
        const double t = td.tbatch[base + (long)j * b + r];
        v = cm_prev<MAXK>(part, nkc, mtot, bmax, slot, r, &t);
      }
      prev[r - (R0 - H)] = v;
      if (r >= R0 && r < R0 + kCmRb) {
        if (FWD) td.tbatch[base + (long)j * b + r] = v;
        else td.batch[base + (long)j * b + r] = v;
      }
    }
    __syncthreads();
  }
  const int r = R0 + threadIdx.x;
  if (r >= b) return;
  const int u1 = r / m0, u0 = r - u1 * m0;
  const int d2 = FWD ? -1 : 1;
  double acc = FWD ? td.batch[base + (long)i * b + r] : 0.0;
  if (couple) {
    const long tn = table_node(g, td.o[0] + u0, td.o[1] + u1, td.o[2] + i);
#pragma unroll
    for (int t9 = 0; t9 < 9; ++t9) {
      const int w0 = u0 + t9 % 3 - 1, w1 = u1 + t9 / 3 - 1;
      if (w0 < 0 || w0 >= m0 || w1 < 0 || w1 >= m1) continue;
      const double c = T[(t9 + 9 * (d2 + 1)) * g.tsize + tn];
      const double v = prev[w0 + m0 * w1 - (R0 - H)];
      acc += FWD ? -c * v : c * v;
    }
  }
  G[(long)slot * bmax + r] = (float)acc;
}

// Partial product of sweep step i: rows [R0, R0 + 128) x the job's members x
// K chunk [K0, K0 + kCmKc) of W_i g, into part[kc][slot][row].
__global__ void __launch_bounds__(kBlock) k_cm_mm(const TypeDev* __restrict__ types,
                                                  const ChainJob* __restrict__ jobs, int i,
                                                  int mtot, int bmax,
                                                  const float* __restrict__ G,
                                                  float* __restrict__ part,
                                                  const PcgState* __restrict__ st) {
  // W_i rows of the chunk [k][row] (row stride kCmLdw); reused for the output
  // tile [row][member] (row stride kCmMembers + 1)
  __shared__ __attribute__((aligned(16))) float ws[kCmKc * kCmLdw];
  __shared__ float gs[kCmKc][kCmMembers + 1];
  if (st != nullptr && st->done) return;
  const ChainJob jb = jobs[blockIdx.z];
  const TypeDev td = types[jb.type];
  const int b = td.b, ldw = td.ldw;
  const int R0 = blockIdx.x * kCmRows, K0 = blockIdx.y * kCmKc;
  if (R0 >= b || K0 >= b) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // W_i through an address-space-1 pointer: its loads are global loads (a flat
  // load would also hold up the LDS wait counter)
  typedef __attribute__((address_space(1))) const f32x4* gvec4;
  const float* Wi = td.W32 + (long)i * b * ldw;
  // W_i rows K0.. of the chunk, columns R0..R0+127 (16-byte loads: ldw and R0
  // are multiples of 4; columns b..ldw-1 of the padded rows are zero), and g
  // of the job's members on the chunk.  All loads are issued before any is
  // used: out-of-range ones read a valid address and are masked afterwards.
  constexpr int NW = (kCmKc * kCmRows / 4) / kBlock, NG = (kCmKc * kCmMembers) / kBlock;
  f32x4 wv[NW];
  float gv[NG];
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int idx = tid + q * kBlock;
    const int k = idx / (kCmRows / 4), col = R0 + 4 * (idx % (kCmRows / 4));
    const bool ok = K0 + k < b && col < ldw;
    wv[q] = *(gvec4)(Wi + (ok ? (long)(K0 + k) * ldw + col : 0));
  }
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int idx = tid + q * kBlock;
    const int j = idx / kCmKc, k = idx % kCmKc;
    const bool ok = j < jb.nm && K0 + k < b;
    gv[q] = G[ok ? (long)(jb.mg0 + j) * bmax + K0 + k : 0];
  }
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int idx = tid + q * kBlock;
    const int k = idx / (kCmRows / 4), c4 = idx % (kCmRows / 4);
    const bool ok = K0 + k < b && R0 + 4 * c4 < ldw;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    *reinterpret_cast<f32x4*>(&ws[k * kCmLdw + 4 * c4]) = ok ? wv[q] : zero;
  }
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int idx = tid + q * kBlock;
    const int j = idx / kCmKc, k = idx % kCmKc;
    gs[k][j] = (j < jb.nm && K0 + k < b) ? gv[q] : 0.0f;
  }
  __syncthreads();
  f32x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
  const int kh = lane >> 5, l32 = lane & 31;
  if (jb.nm > 32) {
#pragma unroll 8
    for (int kk = 0; kk < kCmKc; kk += 2) {
      const float a = ws[(kk + kh) * kCmLdw + w * 32 + l32];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, gs[kk + kh][l32], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, gs[kk + kh][32 + l32], acc[1], 0, 0, 0);
    }
  } else {
#pragma unroll 8
    for (int kk = 0; kk < kCmKc; kk += 2) {
      const float a = ws[(kk + kh) * kCmLdw + w * 32 + l32];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, gs[kk + kh][l32], acc[0], 0, 0, 0);
    }
  }
  __syncthreads();
  // accumulator layout: lane l, element e holds row 8 (e / 4) + 4 (l / 32) + e % 4
  // of the wave's 32 rows and member l % 32 of the tile
  constexpr int LO = kCmMembers + 1;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = w * 32 + 8 * (e >> 2) + 4 * kh + (e & 3);
      ws[row * LO + 32 * t + l32] = acc[t][e];
    }
  __syncthreads();
  for (int idx = tid; idx < kCmMembers * kCmRows; idx += kBlock) {
    const int j = idx / kCmRows, rr = idx % kCmRows;
    if (j < jb.nm && R0 + rr < b)
      part[((long)blockIdx.y * mtot + jb.mg0 + j) * bmax + R0 + rr] = ws[rr * LO + j];
  }
}

// x_0 = t_0 - (partials) after the backward sweep, or x_0 = t_0 = (partials)
// for a chain of one slice.  Grid: (row blocks, jobs, members).
template <int MAXK>
__global__ void __launch_bounds__(kBlock) k_cm_fin(const TypeDev* __restrict__ types,
                                                   const ChainJob* __restrict__ jobs, int mtot,
                                                   int bmax, const float* __restrict__ part,
                                                   const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  const ChainJob jb = jobs[blockIdx.y];
  const int m = blockIdx.z;
  if (m >= jb.nm) return;
  const TypeDev td = types[jb.type];
  const int b = td.b;
  const int nkc = (b + kCmKc - 1) / kCmKc;
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= b) return;
  const long at = (long)(jb.m0 + m) * td.nch * b + r;
  const int slot = jb.mg0 + m;
  if (td.nch == 1) {
    td.batch[at] = cm_prev<MAXK>(part, nkc, mtot, bmax, slot, r, nullptr);
  } else {
    const double t = td.tbatch[at];
    td.batch[at] = cm_prev<MAXK>(part, nkc, mtot, bmax, slot, r, &t);
  }
}

size_t chain_mfma_part_bytes(int bmax, int mtot) {
  const int nkc = (bmax + kCmKc - 1) / kCmKc;
  return (size_t)(nkc + 1) * mtot * bmax * sizeof(float);
}

// The two sweeps over the chain of every class (all classes share nch).
void launch_chain_mfma(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  const int nch = P->types[0].box.nch;
  const int bmax = P->chain_bmax, mtot = P->chain_mtot;
  const int nkc = (bmax + kCmKc - 1) / kCmKc;
  float* part = reinterpret_cast<float*>(P->chain_part);
  float* G = part + (long)nkc * mtot * bmax;
  const dim3 grhs((bmax + kCmRb - 1) / kCmRb, P->nchainjobs, kCmMembers);
  const dim3 gmm((bmax + kCmRows - 1) / kCmRows, nkc, P->nchainjobs);
  const bool k16 = nkc <= 16;
  auto rhs_f = k16 ? k_cm_rhs<true, 16> : k_cm_rhs<true, kCmMaxKc>;
  auto rhs_b = k16 ? k_cm_rhs<false, 16> : k_cm_rhs<false, kCmMaxKc>;
  auto fin = k16 ? k_cm_fin<16> : k_cm_fin<kCmMaxKc>;
  for (int i = 0; i < nch; ++i) {
    hipLaunchKernelGGL(rhs_f, grhs, dim3(kBlock), 0, s, P->g, P->tabAs, P->dTypes,
                       P->dChainJobs, i, mtot, bmax, part, G, st);
    hipLaunchKernelGGL(k_cm_mm, gmm, dim3(kBlock), 0, s, P->dTypes, P->dChainJobs, i, mtot, bmax,
                       G, part, st);
  }
  for (int i = nch - 2; i >= 0; --i) {
    hipLaunchKernelGGL(rhs_b, grhs, dim3(kBlock), 0, s, P->g, P->tabAs, P->dTypes,
                       P->dChainJobs, i, mtot, bmax, part, G, st);
    hipLaunchKernelGGL(k_cm_mm, gmm, dim3(kBlock), 0, s, P->dTypes, P->dChainJobs, i, mtot, bmax,
                       G, part, st);
  }
  const dim3 gfin((bmax + kBlock - 1) / kBlock, P->nchainjobs, kCmMembers);
  hipLaunchKernelGGL(fin, gfin, dim3(kBlock), 0, s, P->dTypes, P->dChainJobs, mtot, bmax, part, st);
}

}  // namespace ddeig

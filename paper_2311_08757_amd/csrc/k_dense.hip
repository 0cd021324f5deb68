// Dense-inverse local solves on MFMA.
//
// All interior subdomains share one local matrix A_sigma,i (the operator is
// periodic and the subdomains are period-aligned), so its inverse is built
// once per subdomain class and the level-1 preconditioner of §3
// (eq:twoLevelASMPreconditioner) applies it to every member of the class at
// once: Z = R Ainv, with R the restricted residuals (one row per subdomain).
// Ainv is symmetric, so the rows of Ainv serve as the columns of the B
// operand and both operands are read row-wise.
//
// Precision: R is split into bf16 pairs r = r_hi + r_lo.  With local_prec = 2
// Ainv is split the same way and Z = R_hi A_hi + R_hi A_lo + R_lo A_hi is
// accumulated in FP32 on v_mfma_f32_32x32x16_bf16 (about 16 significant bits);
// with local_prec = 3 Ainv is a single bf16 (Z = R_hi A + R_lo A, half the
// bytes; the rounded inverse stays positive definite for these local
// matrices, and CG reports a breakdown if it does not).  The extension adds Z
// to the FP64 residual path; the outer CG stays FP64.
//
// Tiling: 128 x 128 output tiles (4 waves of 2 x 2 MFMA tiles), BK = 32 per
// stage with LDS double buffering, split-K partial tiles summed in a fixed
// order by the extension kernel.  Classes with at most kGemvMax members (the
// boundary cells) use a streaming matrix-vector kernel instead.
#include "k_common.h"

namespace ddeig {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int kTK = 32, kLdsK = kTK + 8;

__device__ inline void split_bf16(double x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)(float)x;
  lo = (__bf16)(float)(x - (double)(float)hi);
}

// Ainv (m x m FP64, row-major, from the chain solves of the identity) ->
// symmetrised bf16 hi/lo pairs in an ld x ld zero-padded array.
__global__ void k_split_inverse(const double* __restrict__ Ainv, int m, int ld,
                                __bf16* __restrict__ Ah, __bf16* __restrict__ Al) {
  const long tot = (long)ld * ld;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / ld), j = (int)(idx % ld);
    double v = 0.0;
    if (i < m && j < m) v = 0.5 * (Ainv[(long)i * m + j] + Ainv[(long)j * m + i]);
    __bf16 hi, lo;
    split_bf16(v, hi, lo);
    Ah[idx] = hi;
    if (Al != nullptr) Al[idx] = lo;
  }
}

void launch_split_inverse(const double* Ainv, int m, int ld, void* Ah, void* Al, hipStream_t s) {
  const long tot = (long)ld * ld;
  const int blocks = (int)std::min<long>((tot + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_split_inverse, dim3(blocks), dim3(kBlock), 0, s, Ainv, m, ld,
                     (__bf16*)Ah, (__bf16*)Al);
}

__global__ void k_identity(double* __restrict__ v, int m) {
  const long tot = (long)m * m;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x)
    v[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
}

void launch_identity(double* v, int m, hipStream_t s) {
  const long tot = (long)m * m;
  const int blocks = (int)std::min<long>((tot + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_identity, dim3(blocks), dim3(kBlock), 0, s, v, m);
}

// One 128 x 128 tile of Z (rows: subdomains of one class, columns: local
// unknowns) over the K range [k0, k1) of one split.  4 waves as 2 x 2, each
// owning 2 x 2 MFMA tiles of 32 x 32.  Operands go global -> registers -> LDS
// (double buffered, BK = 32 per stage, rows padded to kLdsK so that the
// 16-byte LDS reads of a wave hit distinct banks).  Each thread moves 32
// bytes of one row of each of R_hi, R_lo, Ainv_hi, Ainv_lo per stage.
constexpr int kTM = 128, kTN = 128;

// ALO: Ainv carries a bf16 lo part (bf16x3 products); without it the inverse
// is a single bf16 and Z = R_hi A + R_lo A (two products, half the bytes).
template <bool ALO>
__global__ void __launch_bounds__(kBlock) k_dense_gemm(const GemmTile* __restrict__ tiles,
                                                       const GemmType* __restrict__ gtypes,
                                                       const PcgState* __restrict__ st) {
  __shared__ __bf16 sA[2][2][kTM * kLdsK];  // [buffer][hi/lo][row * kLdsK + k]  (R rows)
  __shared__ __bf16 sB[2][ALO ? 2 : 1][kTN * kLdsK];  // [buffer][hi/lo][col * kLdsK + k]
  if (st != nullptr && st->done) return;
  const GemmTile t = tiles[blockIdx.x];
  const GemmType gt = gtypes[t.type];
  const int ld = gt.ld;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int lrow = tid >> 1, lhalf = tid & 1;
  const __bf16* gRh = gt.Rh + (long)(t.m0 + lrow) * ld + lhalf * 16;
  const __bf16* gRl = gt.Rl + (long)(t.m0 + lrow) * ld + lhalf * 16;
  const __bf16* gAh = gt.Ah + (long)(t.n0 + lrow) * ld + lhalf * 16;
  const __bf16* gAl = gt.Al + (long)(t.n0 + lrow) * ld + lhalf * 16;
  const int soff = lrow * kLdsK + lhalf * 16;
  typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;
  u32x4 pre[8];
  auto load = [&](int k) {
    pre[0] = *reinterpret_cast<const u32x4*>(gRh + k);
    pre[1] = *reinterpret_cast<const u32x4*>(gRh + k + 8);
    pre[2] = *reinterpret_cast<const u32x4*>(gRl + k);
    pre[3] = *reinterpret_cast<const u32x4*>(gRl + k + 8);
    pre[4] = *reinterpret_cast<const u32x4*>(gAh + k);
    pre[5] = *reinterpret_cast<const u32x4*>(gAh + k + 8);
    if constexpr (ALO) {
      pre[6] = *reinterpret_cast<const u32x4*>(gAl + k);
      pre[7] = *reinterpret_cast<const u32x4*>(gAl + k + 8);
    }
  };
  auto stage = [&](int buf) {
    *reinterpret_cast<u32x4*>(&sA[buf][0][soff]) = pre[0];
    *reinterpret_cast<u32x4*>(&sA[buf][0][soff + 8]) = pre[1];
    *reinterpret_cast<u32x4*>(&sA[buf][1][soff]) = pre[2];
    *reinterpret_cast<u32x4*>(&sA[buf][1][soff + 8]) = pre[3];
    *reinterpret_cast<u32x4*>(&sB[buf][0][soff]) = pre[4];
    *reinterpret_cast<u32x4*>(&sB[buf][0][soff + 8]) = pre[5];
    if constexpr (ALO) {
      *reinterpret_cast<u32x4*>(&sB[buf][ALO ? 1 : 0][soff]) = pre[6];
      *reinterpret_cast<u32x4*>(&sB[buf][ALO ? 1 : 0][soff + 8]) = pre[7];
    }
  };
  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  const int nk = (t.k1 - t.k0) / kTK;
  load(t.k0);
  stage(0);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    if (kb + 1 < nk) load(t.k0 + (kb + 1) * kTK);
#pragma unroll
    for (int ks = 0; ks < kTK / 16; ++ks) {
      const int kof = ks * 16 + 8 * (lane >> 5);
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = (wm * 2 + i) * 32 + (lane & 31);
        ah[i] = *reinterpret_cast<const bf16x8*>(&sA[buf][0][r * kLdsK + kof]);
        al[i] = *reinterpret_cast<const bf16x8*>(&sA[buf][1][r * kLdsK + kof]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = (wn * 2 + j) * 32 + (lane & 31);
        bh[j] = *reinterpret_cast<const bf16x8*>(&sB[buf][0][c * kLdsK + kof]);
        if constexpr (ALO) bl[j] = *reinterpret_cast<const bf16x8*>(&sB[buf][ALO ? 1 : 0][c * kLdsK + kof]);
      }
      // the three products of the split, each over the 4 independent
      // accumulators, so consecutive MFMAs do not wait on each other
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      if constexpr (ALO) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    }
    if (kb + 1 < nk) stage(buf ^ 1);
    __syncthreads();
  }
  // accumulator layout of the 32 x 32 MFMA tile: lane l, element e holds
  // row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
  float* Zp = gt.Z + (long)t.split * gt.zsplit + (long)t.m0 * ld + t.n0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = (wm * 2 + i) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int c = (wn * 2 + j) * 32 + (lane & 31);
        Zp[(long)r * ld + c] = acc[i][j][e];
      }
}

// Classes with at most kGemvMax members (the boundary classes): a streaming
// matrix-vector product, one wave per output row, reading the row of
// Ainv_hi + Ainv_lo once with 16-byte loads and multiplying every member's
// residual (R_hi + R_lo) in FP32.  This is memory-bound on the inverse.
template <bool ALO>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(const GemvRows* __restrict__ jobs,
                                                       const GemmType* __restrict__ gtypes,
                                                       const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  const GemvRows job = jobs[blockIdx.x];
  const GemmType gt = gtypes[job.type];
  const int ld = gt.ld, lane = threadIdx.x & 63;
  const int row = job.r0 + (threadIdx.x >> 6);
  if (row >= job.r1) return;
  typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;
  float acc[kGemvMax];
#pragma unroll
  for (int m = 0; m < kGemvMax; ++m) acc[m] = 0.0f;
  const __bf16* ah = gt.Ah + (long)row * ld;
  const __bf16* al = gt.Al + (long)row * ld;
  for (int k = lane * 8; k < ld; k += 64 * 8) {
    const u32x4 vh = *reinterpret_cast<const u32x4*>(ah + k);
    const __bf16* h = reinterpret_cast<const __bf16*>(&vh);
    float a[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = (float)h[e];
    if constexpr (ALO) {
      const u32x4 vl = *reinterpret_cast<const u32x4*>(al + k);
      const __bf16* l = reinterpret_cast<const __bf16*>(&vl);
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] += (float)l[e];
    }
#pragma unroll
    for (int m = 0; m < kGemvMax; ++m) {
      if (m >= job.nmem) break;
      const u32x4 rh4 = *reinterpret_cast<const u32x4*>(gt.Rh + (long)m * ld + k);
      const u32x4 rl4 = *reinterpret_cast<const u32x4*>(gt.Rl + (long)m * ld + k);
      const __bf16* rh = reinterpret_cast<const __bf16*>(&rh4);
      const __bf16* rl = reinterpret_cast<const __bf16*>(&rl4);
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[m] += a[e] * ((float)rh[e] + (float)rl[e]);
    }
  }
#pragma unroll
  for (int m = 0; m < kGemvMax; ++m) {
    if (m >= job.nmem) break;
    float v = acc[m];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) gt.Z[(long)m * ld + row] = v;
  }
}

// Classes with many members: 128 x 128 MFMA tiles (two workgroups per CU).
void launch_dense_gemm(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  if (P->ntiles > 0) {
    if (P->opt.local_prec == 2)
      hipLaunchKernelGGL(k_dense_gemm<true>, dim3(P->ntiles), dim3(kBlock), 0, s, P->dTiles,
                         P->dGtypes, st);
    else
      hipLaunchKernelGGL(k_dense_gemm<false>, dim3(P->ntiles), dim3(kBlock), 0, s, P->dTiles,
                         P->dGtypes, st);
  }
}

void launch_dense_gemv(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  if (P->ngemv > 0) {
    if (P->opt.local_prec == 2)
      hipLaunchKernelGGL(k_dense_gemv<true>, dim3(P->ngemv), dim3(kBlock), 0, s, P->dGemv,
                         P->dGtypes, st);
    else
      hipLaunchKernelGGL(k_dense_gemv<false>, dim3(P->ngemv), dim3(kBlock), 0, s, P->dGemv,
                         P->dGtypes, st);
  }
}

}  // namespace ddeig

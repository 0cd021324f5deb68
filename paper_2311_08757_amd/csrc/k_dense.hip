// Dense-inverse local solves on MFMA.
//
// Interior subdomains share one local matrix A_sigma,i (the operator is
// periodic and the subdomains are period-aligned), and a subdomain clipped by
// the global boundary has a principal submatrix of it, so one inverse of the
// unclipped box serves the level-1 preconditioner of §3
// (eq:twoLevelASMPreconditioner) for every subdomain: Z = R Ainv with R the
// restricted residuals (one row per subdomain), followed by a small
// Schur-complement correction for the clipped ones.  Ainv is symmetric, so
// its rows serve as the columns of the B operand and both operands are read
// row-wise.
//
// Precision: with local_prec = 2 the residual and Ainv are split into bf16
// pairs x = x_hi + x_lo and Z = R_hi A_hi + R_hi A_lo + R_lo A_hi is
// accumulated in FP32 on v_mfma_f32_32x32x16_bf16 (about 16 significant bits).
// With local_prec = 3 both are single bf16 and Z = R A (one product; the
// rounded inverse stays positive definite for these local matrices, and CG
// reports a breakdown if it does not).  Rounding the residual makes the
// preconditioner vary slightly between iterations (relative 2^-9); the outer
// CG is FP64 and its residual is updated by the exact recurrence, so this
// changes the iteration count a little, not the attainable accuracy.  The
// extension adds Z to the FP64 residual path.
//
// Tiling: 128 x 128 output tiles (4 waves of 2 x 2 MFMA tiles), or 64 x 128
// (4 waves of 1 x 2; batches choose them where instances have few subdomain
// rows, to skip padding rows), 64 (bf16) or 32 (bf16x3) K columns per stage,
// two stages of global loads in flight and LDS double buffering, split-K
// partial tiles summed in a fixed order by the extension kernel.  Classes with at most kGemvMax members (the
// boundary cells) use a streaming matrix-vector kernel instead.
#include "k_common.h"
#include "k_coarse.h"

namespace ddeig {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;


__device__ inline void split_bf16(double x, __bf16& hi, __bf16& lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - (double)hi);
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
// in stages of BK columns of K (LDS double buffered, rows padded to BK + 8 so
// that the 16-byte fragment reads of a wave spread over the banks):
//  - the global loads of stage s + 2 are issued before the MFMAs of stage s,
//    so two stages of loads are in flight while the matrix cores work;
//  - inside a stage the fragments of MFMA sub-step j + 1 are read from LDS
//    and a share of stage s + 1's registers is written to the other LDS
//    buffer while the MFMAs of sub-step j run.
// Operands: R_hi, R_lo (RLO), A_hi, A_lo (ALO).
constexpr int kTM = 128, kTN = 128;

template <bool RLO, bool ALO, int MI>
struct GemmCfg {
  static constexpr int BK = (RLO && ALO) ? 32 : 64;  // K columns per stage
  static constexpr int LDK = BK + 8;                 // padded LDS row
  static constexpr int NR = RLO ? 2 : 1, NA = ALO ? 2 : 1;
  static constexpr int NOP = NR + NA;                // operands staged per stage
  static constexpr int TM = 64 * MI;                 // rows of the tile (R operand)
  static constexpr int NV = BK / 16;                 // 16-byte vectors per thread, A operand
  static constexpr int NVR = NV * MI / 2;            // 16-byte vectors per thread, R operand
  static constexpr int NVT = NR * NVR + NA * NV;     // vectors per thread per stage
  static constexpr int NS = BK / 16;                 // MFMA sub-steps per stage
  static constexpr int WPS = (NVT + NS - 1) / NS;    // vectors staged per sub-step
};

typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

// Workgroups beyond the ntiles tiles form the coarse right-hand side R_0 r
// (ca.n of them, one per subdomain) on the CUs the tiles leave free; they
// share nothing with the tiles, so no workgroup waits for another.
template <bool RLO, bool ALO, int MI = 2, bool BND = false>
__global__ void __launch_bounds__(kBlock) k_dense_gemm(const GemmTile* __restrict__ tiles,
                                                       const GemmType* __restrict__ gtypes,
                                                       const PcgState* __restrict__ st,
                                                       int ntiles, CoarseRhsArgs ca) {
  using C = GemmCfg<RLO, ALO, MI>;
  constexpr int BK = C::BK, LDK = C::LDK, NR = C::NR, NOP = C::NOP, NV = C::NV, NVT = C::NVT;
  constexpr int NVR = C::NVR, NS = C::NS, WPS = C::WPS;
  static_assert(MI == 1 || MI == 2, "64- or 128-row tiles");
  // [buffer][operand][row * LDK + k]; operands: R parts first, then A parts
  __shared__ __bf16 sm[2][NOP][kTM * LDK];
  if (st != nullptr && st->done) return;
  if ((int)blockIdx.x >= ntiles) {
    coarse_rhs_body(ca.g, nullptr, ca.r, ca.types, ca.subs, ca.crhs, blockIdx.x - ntiles);
    return;
  }
  const GemmTile t = tiles[blockIdx.x];
  const GemmType gt = gtypes[t.type];
  if (gt.st != nullptr && gt.st->done) return;
  const int ld = gt.ld;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  // loader: A operand row tid / 2, half tid % 2 of the BK columns of a stage;
  // R operand (TM rows) row tid / (256 / TM), the matching share of the
  // columns.  The operands live in global memory: loads through
  // address-space-1 pointers become global_load (flat loads would also count
  // against the LDS wait counter and stall every fragment read behind the
  // prefetch).
  typedef __attribute__((address_space(1))) const u32x4* gvec;
  const int lrow = tid >> 1, lcol = (tid & 1) * (BK / 2);
  constexpr int RPT = kBlock / C::TM;  // threads per R row
  static_assert(RPT * C::TM == kBlock && (BK / RPT) % 8 == 0, "whole vectors per thread");
  const int rrow = tid / RPT, rcol = (tid % RPT) * (BK / RPT);
  gvec gsrc[NOP];
  gsrc[0] = (gvec)(gt.Rh + (long)(t.m0 + rrow) * ld + rcol);
  if constexpr (RLO) gsrc[1] = (gvec)(gt.Rl + (long)(t.m0 + rrow) * ld + rcol);
  gsrc[NR] = (gvec)(gt.Ah + (long)(t.n0 + lrow) * ld + lcol);
  if constexpr (ALO) gsrc[NR + 1] = (gvec)(gt.Al + (long)(t.n0 + lrow) * ld + lcol);
  // BND (batches, whose instances leave tile rows unused): R through buffer
  // resources that end at the instance's last subdomain row, so that padding
  // rows read as zero without a memory request (the rows hold zeros), and the
  // padding rows of Z are not stored
  __amdgpu_buffer_rsrc_t rsrc[NR];
  unsigned roff = 0;
  if constexpr (BND) {
    const int rbytes = gt.rows * ld * 2;
    rsrc[0] = __builtin_amdgcn_make_buffer_rsrc((void*)gt.Rh, (short)0, rbytes, 0x00020000);
    if constexpr (RLO)
      rsrc[1] = __builtin_amdgcn_make_buffer_rsrc((void*)gt.Rl, (short)0, rbytes, 0x00020000);
    roff = (unsigned)(((t.m0 + rrow) * ld + rcol) * 2);
  }
  const int soff = lrow * LDK + lcol, sroff = rrow * LDK + rcol;
  u32x4 ra[NVT], rb[NVT];
  // vector q of a stage: operand and vector within the operand (R operands
  // first, NVR vectors each, then the A operands, NV each)
  auto qop = [](int q) { return q < NR * NVR ? q / NVR : NR + (q - NR * NVR) / NV; };
  auto qv = [](int q) { return q < NR * NVR ? q % NVR : (q - NR * NVR) % NV; };
  // k: first K column of the stage; 8 bf16 per vector
  auto load = [&](u32x4* dst, int k) {
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      if constexpr (BND) {
        const int o = qop(q);
        if (o < NR) {
          dst[q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                 rsrc[o], roff + 16u * qv(q), (unsigned)k * 2u, 0));
          continue;
        }
      }
      dst[q] = gsrc[qop(q)][k / 8 + qv(q)];
    }
  };
  auto stage1 = [&](const u32x4* src, int buf, int q) {
    if (q < NVT) {
      const int o = qop(q);
      *reinterpret_cast<u32x4*>(&sm[buf][o][(o < NR ? sroff : soff) + 8 * qv(q)]) = src[q];
    }
  };
  struct Frag {
    bf16x8 rh[MI], rl[MI], ah[2], al[2];
  };
  auto rd = [&](Frag& f, int buf, int ks) {
    const int kof = ks * 16 + 8 * (lane >> 5);
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int r = (wm * MI + i) * 32 + (lane & 31);
      f.rh[i] = *reinterpret_cast<const bf16x8*>(&sm[buf][0][r * LDK + kof]);
      if constexpr (RLO) f.rl[i] = *reinterpret_cast<const bf16x8*>(&sm[buf][1][r * LDK + kof]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = (wn * 2 + j) * 32 + (lane & 31);
      f.ah[j] = *reinterpret_cast<const bf16x8*>(&sm[buf][NR][c * LDK + kof]);
      if constexpr (ALO) f.al[j] = *reinterpret_cast<const bf16x8*>(&sm[buf][NR + 1][c * LDK + kof]);
    }
  };
  floatx16 acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  // the products of the split, small parts first, each over the 4 independent
  // accumulators so that consecutive MFMAs do not wait on each other
  auto mm = [&](const Frag& f) {
    if constexpr (RLO) {
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.rl[i], f.ah[j], acc[i][j], 0, 0, 0);
    }
    if constexpr (ALO) {
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.rh[i], f.al[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.rh[i], f.ah[j], acc[i][j], 0, 0, 0);
  };
  // stages of the K range; the host splits K into an even number of stages
  const int nk = (t.k1 - t.k0) / BK;
  load(ra, t.k0);
  load(rb, t.k0 + BK);
#pragma unroll
  for (int q = 0; q < NVT; ++q) stage1(ra, 0, q);
  __syncthreads();
  // stage kb from LDS buffer `buf`: loads of kb + 2 into the register set
  // staged last, writes of kb + 1 into the other buffer spread over the
  // sub-steps.  Loads and stores are unconditional (past the end the last
  // stage is loaded again and staged into a buffer nobody reads), so the loop
  // body has no branches and the compiler's load counters stay exact; the
  // scheduling barriers keep the compiler from regrouping the three streams.
  auto half = [&](u32x4* ld_dst, const u32x4* st_src, int buf, int kb) {
    load(ld_dst, t.k0 + min(kb + 2, nk - 1) * BK);
    Frag f[2];
    rd(f[0], buf, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < NS; ++ks) {
      if (ks + 1 < NS) rd(f[(ks + 1) & 1], buf, ks + 1);
#pragma unroll
      for (int q = 0; q < WPS; ++q) stage1(st_src, buf ^ 1, ks * WPS + q);
      __builtin_amdgcn_sched_barrier(0);
      mm(f[ks & 1]);
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  };
  for (int kb = 0; kb < nk; kb += 2) {
    half(ra, rb, 0, kb);
    half(rb, ra, 1, kb + 1);
  }
  // accumulator layout of the 32 x 32 MFMA tile: lane l, element e holds
  // row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
  float* Zp = gt.Z + (long)t.split * gt.zsplit + (long)t.m0 * ld + t.n0;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = (wm * MI + i) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int c = (wn * 2 + j) * 32 + (lane & 31);
        if (!BND || t.m0 + r < gt.rows) Zp[(long)r * ld + c] = acc[i][j][e];
      }
}

// Batches of at most kGemvMax rows (domains of at most kGemvMax cells): a
// streaming matrix-vector product, one wave per output row, reading the row
// of Ainv_hi (+ Ainv_lo) once with 16-byte loads and multiplying every
// member's residual (R_hi (+ R_lo)) in FP32.  This is memory-bound on the
// inverse.
template <bool RLO, bool ALO>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(const GemvRows* __restrict__ jobs,
                                                       const GemmType* __restrict__ gtypes,
                                                       const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  const GemvRows job = jobs[blockIdx.x];
  const GemmType gt = gtypes[job.type];
  const int ld = gt.ld, lane = threadIdx.x & 63;
  const int row = job.r0 + (threadIdx.x >> 6);
  if (row >= job.r1) return;
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
      const __bf16* rh = reinterpret_cast<const __bf16*>(&rh4);
      float rv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) rv[e] = (float)rh[e];
      if constexpr (RLO) {
        const u32x4 rl4 = *reinterpret_cast<const u32x4*>(gt.Rl + (long)m * ld + k);
        const __bf16* rl = reinterpret_cast<const __bf16*>(&rl4);
#pragma unroll
        for (int e = 0; e < 8; ++e) rv[e] += (float)rl[e];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[m] += a[e] * rv[e];
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

// Clipped classes.  The local matrix of a subdomain clipped by the global
// boundary is the principal submatrix A_SS of the unclipped box's matrix A
// (the operator is periodic and the clipped box keeps the unclipped node
// positions), and for B = A^{-1} the Schur-complement identity gives
// (A_SS)^{-1} = B_SS - B_ST (B_TT)^{-1} B_TS.  The batch row of a clipped
// member holds r_S and zeros on T, so the GEMM returns u = B [r_S; 0]; the
// correction then forms y_S = u_S - G u_T with G = B_ST (B_TT)^{-1}, built
// once per shift.  With the rounded
// inverse B~ in place of B this is exactly the Schur complement of B~, which
// stays symmetric positive definite whenever B~ is.

// B~_TT of a clipped class (hi + lo parts), FP64, row-major nT x nT.
__global__ void k_embed_gather(const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al,
                               int ld, const int* __restrict__ Tidx, int nT,
                               double* __restrict__ C) {
  const long tot = (long)nT * nT;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / nT), j = (int)(idx % nT);
    const long a = (long)Tidx[i] * ld + Tidx[j];
    double v = (double)(float)Ah[a];
    if (Al != nullptr) v += (double)(float)Al[a];
    C[idx] = v;
  }
}

void launch_embed_gather(const ddeig_problem* P, const EmbedDev& E, double* C, hipStream_t s) {
  const long tot = (long)E.nT * E.nT;
  const int blocks = (int)std::min<long>((tot + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_embed_gather, dim3(blocks), dim3(kBlock), 0, s, P->dh.Ah, P->dh.Al,
                     P->dh.ld, E.Tidx, E.nT, C);
}

// Set-up: G = B~_ST (B~_TT)^{-1}, t-major over the unclipped box, zero for
// the nodes in T; one thread per entry, FP64 sums in index order.
__device__ inline bool embed_in_box(const EmbedDev& E, int e, int hm0, int hm1) {
  const int u0 = e % hm0, rest = e / hm0;
  const int u1 = rest % hm1, u2 = rest / hm1;
  return u0 >= E.off[0] && u0 < E.off[0] + E.m[0] && u1 >= E.off[1] && u1 < E.off[1] + E.m[1] &&
         u2 >= E.off[2] && u2 < E.off[2] + E.m[2];
}

__global__ void k_embed_gmat(EmbedDev E, const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al,
                             int ld, int hm0, int hm1, int mH, const double* __restrict__ C,
                             float* __restrict__ G) {
  const long tot = (long)E.nT * mH;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int t = (int)(idx / mH), e = (int)(idx % mH);
    double v = 0.0;
    if (embed_in_box(E, e, hm0, hm1)) {
      for (int j = 0; j < E.nT; ++j) {
        const long a = (long)e * ld + E.Tidx[j];
        double b = (double)(float)Ah[a];
        if (Al != nullptr) b += (double)(float)Al[a];
        v += b * C[(long)j * E.nT + t];
      }
    }
    G[idx] = (float)v;
  }
}

void launch_embed_gmat(const ddeig_problem* P, const EmbedDev& E, const double* C, float* G,
                       hipStream_t s) {
  const DenseHost& H = P->dh;
  const long tot = (long)E.nT * H.m;
  const int blocks = (int)std::min<long>((tot + kBlock - 1) / kBlock, 16384);
  hipLaunchKernelGGL(k_embed_gmat, dim3(blocks), dim3(kBlock), 0, s, E, H.Ah, H.Al, H.ld,
                     H.box.m[0], H.box.m[1], H.m, C, G);
}

// Per application: y_S = u_S - G u_T for the members of one job of a class
// (at most kEmbChunk), u = B~ [r_S; 0] the GEMM result (split-K partials added
// in split order).  The corrected solution replaces split 0 of Z and the other
// splits are cleared, so the extension reads clipped and unclipped members
// alike.
// Block (64 unknowns of the unclipped box, job): thread (unknown, phase) adds
// the terms t = phase mod 4 in batches of kEmbG for every member (a wave reads
// 256 contiguous bytes of a row of G per load); the 4 phase sums of a member
// are added in phase order by the thread of phase m mod 4.
// u_T sits in LDS with the members of one t next to each other (two 16-byte
// reads per term).  The first batch of the thread's column of G and its
// members' own Z entries are loaded before u_T is gathered (kEmbGU values per
// thread in flight), and each later batch of G is loaded while the previous
// one is used.  Nodes in T are left alone (no member reads them).
constexpr int kEmbPh = 4, kEmbE = kBlock / kEmbPh, kEmbG = 32;  // G loads per batch
constexpr int kEmbGU = 8;                                         // gather depth
constexpr int kEmbOwn = kEmbChunk / kEmbPh;                        // members finished per thread
static_assert(kEmbChunk % kEmbPh == 0, "members are finished round-robin over the phases");
static_assert(kEmbChunk == 8 && kEmbUT == kEmbMaxT * kEmbChunk,
              "u_T rows are two float4 of members, for every t < kEmbMaxT");

// The terms of one thread for NM members: gv holds the first batch of G on
// entry (G[g0 + q gs], q < nq, is the thread's column; nT mH < 2^31 is checked
// at set-up); each register is refilled with its term of the next batch as
// soon as it has been used.
template <int NM>
__device__ __forceinline__ void embed_accumulate(const float* __restrict__ G, unsigned g0,
                                                 unsigned gs, int nq,
                                                 const float* __restrict__ uT, int ph,
                                                 float (&gv)[kEmbG], float (&acc)[kEmbChunk]) {
  for (int q0 = 0; q0 < nq; q0 += kEmbG) {
#pragma unroll
    for (int q = 0; q < kEmbG; ++q) {
      const float g = gv[q];
      if (q0 + kEmbG + q < nq) gv[q] = G[g0 + (unsigned)(q0 + kEmbG + q) * gs];
      if (q0 + q < nq) {
        const float4* u4 =
            reinterpret_cast<const float4*>(uT + (ph + kEmbPh * (q0 + q)) * kEmbChunk);
        const float4 a = u4[0];
        float u[kEmbChunk] = {a.x, a.y, a.z, a.w, 0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (NM > 4) {
          const float4 b = u4[1];
          u[4] = b.x; u[5] = b.y; u[6] = b.z; u[7] = b.w;
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[m] += g * u[m];
      }
    }
  }
}

// Grid (row chunk, job): the chunks of one job are consecutive in dispatch
// order, so the blocks that run together read neighbouring pieces of the same
// rows of G.  Chunks blockIdx.x >= ceil(mH / kEmbE) of job 0 apply the coarse
// inverse instead (rows 4 (blockIdx.x - ychunks) .. + 3 of y0 = A_0^{-1} c),
// independent of the correction workgroups.
template <int KS>
// At most 128 VGPRs (4 waves per SIMD, as many as the LDS allows): with more
// the compiler hoists LDS reads and the kernel runs at 3 waves, markedly slower.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_embed_correct(const EmbedJob* __restrict__ jobs, const EmbedDev* __restrict__ cls, int ld,
                int hm0, int hm1, int mH, const PcgState* __restrict__ st, CoarseSolveArgs cs) {
  __shared__ __align__(16) float uT[kEmbUT];  // uT[t kEmbChunk + m] = u_T of member m
  __shared__ float red[kEmbPh][kEmbE][kEmbChunk];
  const int ychunks = (mH + kEmbE - 1) / kEmbE;
  if ((int)blockIdx.x >= ychunks) {
    if (blockIdx.y == 0) coarse_solve_body(cs.n, st, cs.A0inv, cs.c, cs.y, blockIdx.x - ychunks);
    return;
  }
  // the job, the state and the class are loaded before the state is tested,
  // so that their latencies overlap
  const EmbedJob jb = jobs[blockIdx.y];
  const int done0 = st != nullptr ? st->done : 0;
  const EmbedDev E = cls[jb.cls];
  if (done0) return;
  if (E.st != nullptr && E.st->done) return;
  float* __restrict__ Z = E.Z;
  const long zsplit = E.zsplit;
  const int el = threadIdx.x % kEmbE, ph = threadIdx.x / kEmbE;
  const int e = blockIdx.x * kEmbE + el;
  const bool inS = e < mH && embed_in_box(E, e, hm0, hm1);
  const int nq = (E.nT - ph + kEmbPh - 1) / kEmbPh;  // terms t = ph + kEmbPh q, q < nq
  const float* __restrict__ G = E.G;
  const unsigned g0 = (unsigned)(ph * mH + e), gs = (unsigned)(kEmbPh * mH);  // G[g0 + q gs]
  float gv[kEmbG];
  float zown[kEmbOwn][KS];
  if (inS) {
#pragma unroll
    for (int q = 0; q < kEmbG; ++q)
      if (q < nq) gv[q] = G[g0 + (unsigned)q * gs];
#pragma unroll
    for (int k = 0; k < kEmbOwn; ++k) {
      const int m = ph + kEmbPh * k;
      if (m < jb.nm) {
        const long base = (long)E.rows[jb.mem0 + m] * ld + e;
#pragma unroll
        for (int sp = 0; sp < KS; ++sp) zown[k][sp] = Z[sp * zsplit + base];
      }
    }
  }
  const int nmiss = hm0 - E.m[0];
  const int tot = jb.nm * E.nT;  // gather index m nT + t
  for (int i0 = 0; i0 < tot; i0 += kBlock * kEmbGU) {
    float v[kEmbGU];
#pragma unroll
    for (int g = 0; g < kEmbGU; ++g) {
      const int idx = i0 + g * kBlock + threadIdx.x;
      v[g] = 0.0f;
      if (idx < tot) {
        const int m = idx / E.nT, t = idx - m * E.nT;
        int te;
        if (E.xonly) {
          const int line = t / nmiss, j = t - line * nmiss;
          te = (j < E.off[0] ? j : j + E.m[0]) + hm0 * line;
        } else {
          te = E.Tidx[t];
        }
        const long base = (long)E.rows[jb.mem0 + m] * ld + te;
#pragma unroll
        for (int sp = 0; sp < KS; ++sp) v[g] += Z[sp * zsplit + base];
      }
    }
#pragma unroll
    for (int g = 0; g < kEmbGU; ++g) {
      const int idx = i0 + g * kBlock + threadIdx.x;
      if (idx < tot) {
        const int m = idx / E.nT;
        uT[(idx - m * E.nT) * kEmbChunk + m] = v[g];
      }
    }
  }
  __syncthreads();
  float acc[kEmbChunk];
#pragma unroll
  for (int m = 0; m < kEmbChunk; ++m) acc[m] = 0.0f;
  if (inS) {
    switch (jb.nm) {  // 1 <= nm <= kEmbChunk by construction of the jobs
      case 1: embed_accumulate<1>(G, g0, gs, nq, uT, ph, gv, acc); break;
      case 2: embed_accumulate<2>(G, g0, gs, nq, uT, ph, gv, acc); break;
      case 3: embed_accumulate<3>(G, g0, gs, nq, uT, ph, gv, acc); break;
      case 4: embed_accumulate<4>(G, g0, gs, nq, uT, ph, gv, acc); break;
      case 5: embed_accumulate<5>(G, g0, gs, nq, uT, ph, gv, acc); break;
      case 6: embed_accumulate<6>(G, g0, gs, nq, uT, ph, gv, acc); break;
      case 7: embed_accumulate<7>(G, g0, gs, nq, uT, ph, gv, acc); break;
      default: embed_accumulate<8>(G, g0, gs, nq, uT, ph, gv, acc); break;
    }
  }
#pragma unroll
  for (int m = 0; m < kEmbChunk; ++m) red[ph][el][m] = acc[m];
  __syncthreads();
  if (!inS) return;
#pragma unroll
  for (int k = 0; k < kEmbOwn; ++k) {
    const int m = ph + kEmbPh * k;
    if (m >= jb.nm) break;
    float corr = 0.0f;
    for (int q = 0; q < kEmbPh; ++q) corr += red[q][el][m];
    float u = 0.0f;
#pragma unroll
    for (int sp = 0; sp < KS; ++sp) u += zown[k][sp];
    const long base = (long)E.rows[jb.mem0 + m] * ld + e;
    Z[base] = u - corr;
#pragma unroll
    for (int sp = 1; sp < KS; ++sp) Z[sp * zsplit + base] = 0.0f;
  }
}

// With coarse_solve the launch also applies A_0^{-1} to the coarse right-hand
// side (P->crhs into P->cy).
void launch_embed_fix(const ddeig_problem* P, const PcgState* st, hipStream_t s,
                      bool coarse_solve) {
  if (P->nembjobs == 0) return;
  const DenseHost& H = P->dh;
  // the K split is 1..3 by construction (assemble)
  auto kern = P->ksplit == 1 ? k_embed_correct<1> : (P->ksplit == 2 ? k_embed_correct<2>
                                                                     : k_embed_correct<3>);
  CoarseSolveArgs cs{0, nullptr, nullptr, nullptr};
  int extra = 0;
  if (coarse_solve) {
    cs = CoarseSolveArgs{P->nsub, P->A0inv, P->crhs, P->cy};
    extra = (P->nsub + kBlock / 64 - 1) / (kBlock / 64);
  }
  hipLaunchKernelGGL(kern, dim3((H.m + kEmbE - 1) / kEmbE + extra, P->nembjobs), dim3(kBlock), 0,
                     s, P->dEmbJobs, P->dEmb, H.ld, H.box.m[0], H.box.m[1], H.m, st, cs);
}

// Batches of more rows: 128 x 128 MFMA tiles.  local_prec 2 (bf16x3):
// residual and inverse as hi/lo pairs, three products; local_prec 3: both
// single bf16, one product.  coarse_r (nullable): one more workgroup per
// subdomain forms R_0 coarse_r into P->crhs.
void launch_dense_gemm(const ddeig_problem* P, const PcgState* st, hipStream_t s,
                       const double* coarse_r) {
  if (P->ntiles > 0) {
    CoarseRhsArgs ca{};
    ca.n = 0;
    if (coarse_r != nullptr)
      ca = CoarseRhsArgs{P->nsub, P->g, coarse_r, P->dTypes, P->dSubs, P->crhs};
    const dim3 grid(P->ntiles + ca.n);
    if (P->opt.local_prec == 2)
      hipLaunchKernelGGL((k_dense_gemm<true, true>), grid, dim3(kBlock), 0, s, P->dTiles,
                         P->dGtypes, st, P->ntiles, ca);
    else
      hipLaunchKernelGGL((k_dense_gemm<false, false>), grid, dim3(kBlock), 0, s, P->dTiles,
                         P->dGtypes, st, P->ntiles, ca);
  }
}

// The coarse space rides in the GEMM and correction launches (and the coarse
// field is formed inside the extension) when the dense path has both.
bool fused_coarse(const ddeig_problem* P) {
  return P->opt.coarse && P->opt.local_prec >= 2 && P->ntiles > 0 && P->nembjobs > 0;
}

// Grouped launches over the instances of a batch: the tiles / correction jobs
// carry the instance in their type / class index, and each instance's CG
// state is checked through GemmType::st / EmbedDev::st.
void launch_gemm_tiles(const GemmTile* tiles, int ntiles, const GemmType* gt, int local_prec,
                       hipStream_t s, int tile_rows) {
  if (ntiles <= 0) return;
  CoarseRhsArgs none{};
  none.n = 0;
  auto kern = local_prec == 2 ? (tile_rows == 64 ? k_dense_gemm<true, true, 1, true>
                                                 : k_dense_gemm<true, true, 2, true>)
                              : (tile_rows == 64 ? k_dense_gemm<false, false, 1, true>
                                                 : k_dense_gemm<false, false, 2, true>);
  hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kBlock), 0, s, tiles, gt, nullptr, ntiles, none);
}

void launch_embed_jobs(const EmbedJob* jobs, int njobs, const EmbedDev* cls, int ksplit, int ld,
                       int hm0, int hm1, int mH, hipStream_t s) {
  if (njobs <= 0) return;
  auto kern = ksplit == 1 ? k_embed_correct<1> : (ksplit == 2 ? k_embed_correct<2>
                                                               : k_embed_correct<3>);
  const CoarseSolveArgs none{0, nullptr, nullptr, nullptr};
  hipLaunchKernelGGL(kern, dim3((mH + kEmbE - 1) / kEmbE, njobs), dim3(kBlock), 0, s, jobs, cls,
                     ld, hm0, hm1, mH, nullptr, none);
}

void launch_dense_gemv(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  if (P->ngemv > 0) {
    if (P->opt.local_prec == 2)
      hipLaunchKernelGGL((k_dense_gemv<true, true>), dim3(P->ngemv), dim3(kBlock), 0, s, P->dGemv,
                         P->dGtypes, st);
    else
      hipLaunchKernelGGL((k_dense_gemv<false, false>), dim3(P->ngemv), dim3(kBlock), 0, s,
                         P->dGemv, P->dGtypes, st);
  }
}

}  // namespace ddeig

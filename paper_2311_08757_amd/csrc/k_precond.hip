// Restriction, extension and coarse space of the two-level additive Schwarz
// preconditioner (§2.2 eq:dd-preconditioners, eq:two-level-preconditioners,
// §2.3 def:algebraic-perfact-coarse-space, §3 eq:twoLevelASMPreconditioner).
//
// Subdomains are the L^p unit cells extended by delta element layers in every
// expanding direction (§3, §4.1): along an expanding axis, cell c (1-based)
// owns the node indices [(c-1) n_e - delta + 1, c n_e + delta - 1] clipped to
// [1, L n_e - 1]; fixed directions are not split.  With 2 delta <= n_e a node
// lies in at most two cells per axis.  The extension sums, for every node, the
// local solutions of the subdomains covering it in a fixed order (no atomics).
#include "k_common.h"
#include "k_coarse.h"

namespace ddeig {

// 1-based cells covering node index gi (1-based) along one expanding axis.
__device__ inline void covering(int gi, int ne, int L, int delta, int& clo, int& chi) {
  // g <= c ne + delta - 1  <=>  c >= (g - delta + 1) / ne
  const int num = gi - delta + 1;
  clo = num <= 0 ? 1 : (num + ne - 1) / ne;
  chi = (gi + delta - 1) / ne + 1;
  if (clo < 1) clo = 1;
  if (chi > L) chi = L;
}

// Distance from node coordinate (index gi, in units of h) to the faces of
// cell c's box along one axis that are not on the global boundary; INT_MAX if none.
__device__ inline int face_dist(int gi, int c, int ne, int L, int delta) {
  int dmin = 0x7fffffff;
  if (c > 1) {
    const int lo = (c - 1) * ne - delta;  // face at ((c-1) n_e - delta) h
    dmin = min(dmin, gi - lo);
  }
  if (c < L) {
    const int hi = c * ne + delta;
    dmin = min(dmin, hi - gi);
  }
  return dmin;
}

// Partition-of-unity weight of subdomain with cell index c at the node with
// 0-based unknown indices i.  pu = 0: 1 / #covering subdomains (§2.2);
// pu = 1: distance-based d_c / sum_c' d_c' (§4.1.2) with the distance to the
// interior faces of the box (the minimum over axes of perpendicular distances).
__device__ inline double pu_weight(const Geo& g, int delta, int pu, const int* c, const int* i) {
  if (pu == 0) {
    double w = 1.0;
    for (int a = 0; a < g.p; ++a) {
      int clo, chi;
      covering(i[a] + 1, g.ne, g.L, delta, clo, chi);
      w /= (double)(chi - clo + 1);
    }
    return w;
  }
  int lo[2] = {1, 1}, hi[2] = {1, 1};
  for (int a = 0; a < g.p; ++a) covering(i[a] + 1, g.ne, g.L, delta, lo[a], hi[a]);
  auto dist = [&](const int* cc) {
    int dm = 0x7fffffff;
    for (int a = 0; a < g.p; ++a) dm = min(dm, face_dist(i[a] + 1, cc[a], g.ne, g.L, delta));
    return dm;
  };
  const int dc = dist(c);
  if (dc == 0x7fffffff) return 1.0;  // a single subdomain: no interior faces
  double tot = 0.0;
  for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
    for (int c0 = lo[0]; c0 <= hi[0]; ++c0) {
      const int cc[2] = {c0, c1};
      tot += (double)dist(cc);
    }
  return (double)dc / tot;
}

__device__ inline int sub_index(const Geo& g, const int* c) {
  return g.p == 1 ? c[0] - 1 : (c[0] - 1) + g.L * (c[1] - 1);
}

// Partition-of-unity weight of cell c at a node from the per-axis covering
// tables: the product of the per-axis factors, except for the distance-based
// weights with two expanding axes, which are not separable (pu_weight).
__device__ inline double cover_weight(const Geo& g, int delta, int pu, const XCover* const* xc,
                                      const int* c, const int* i, const int* which) {
  if (pu == 1 && g.p == 2) return pu_weight(g, delta, pu, c, i);
  double w = xc[0][i[0]].w[which[0]];
  if (g.p == 2) w *= xc[1][i[1]].w[which[1]];
  return w;
}

// Scatter r into the subdomain batches (box natural order; bf16 rows, as a
// hi/lo pair for local_prec 2, for dense classes): node-parallel over row
// segments of kBlock x1 positions, four segments per workgroup of kBig
// threads (one node per thread, so the dependent table loads of the nodes
// overlap); every node writes its copy into each covering subdomain (at most
// 2^p), so reads of r and writes of a batch row are both coalesced.  With
// xr.on the node first takes the CG update of iteration k (x += alpha p,
// r -= alpha q, written back) and the kernel leaves the partials of ||r||^2
// in rr.
__global__ void __launch_bounds__(kBig) k_restrict(Geo g, int ntypes, PcgState* __restrict__ st,
                                                   XrArgs xr, Red rr, double* __restrict__ r,
                                                   const TypeDev* __restrict__ types,
                                                   const SubTS* __restrict__ subts,
                                                   const XCover* __restrict__ xc0,
                                                   const XCover* __restrict__ xc1) {
  __shared__ TypeDev stypes[kMaxTypes];
  if (st != nullptr && st->done) return;
  double alpha = 0.0;
  if (xr.on == 1) {
    const double gamma = sum_partials<kBig>(xr.gam.part, xr.gam.np);
    if (!(gamma > 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 2;
        st->iters = xr.k - 1;
      }
      return;
    }
    alpha = st->rho[(xr.k - 1) & 1] / gamma;
  }
  if (threadIdx.x < ntypes) stypes[threadIdx.x] = types[threadIdx.x];
  __syncthreads();
  const int N0 = g.N[0], N1 = g.N[1];
  const int segs = (N0 + kBlock - 1) / kBlock;
  const long items = (long)segs * N1 * g.N[2];
  const int sub = threadIdx.x / kBlock, tx = threadIdx.x % kBlock;
  double acc = 0.0;
  for (long grp = blockIdx.x; grp * (kBig / kBlock) < items; grp += gridDim.x) {
    const long it = grp * (kBig / kBlock) + sub;
    if (it >= items) continue;
    const int line = (int)(it / segs);
    const int i0 = (int)(it - (long)line * segs) * kBlock + tx;
    if (i0 >= N0) continue;
    const int i2 = g.D == 3 ? (int)fdiv((unsigned)line, g.fN1) : 0;
    const int i1 = line - i2 * N1;
    const long k = i0 + (long)N0 * line;
    double rv = r[k];
    if (xr.on) {
      rv -= alpha * xr.q[k];
      xr.x[k] += alpha * xr.p[k];
      r[k] = rv;
      acc += rv * rv;
    }
    const __bf16 hi = to_bf16(rv);
    const __bf16 lo = to_bf16(rv - (double)hi);
    const XCover a0 = xc0[i0];
    XCover a1;
    a1.c[0] = 1; a1.c[1] = 0; a1.u[0] = i1; a1.u[1] = 0;
    if (g.p == 2) a1 = xc1[i1];
    for (int q1 = 0; q1 < 2; ++q1) {
      if (a1.c[q1] == 0) continue;
      for (int q0 = 0; q0 < 2; ++q0) {
        if (a0.c[q0] == 0) continue;
        const int sid = g.p == 1 ? a0.c[q0] - 1 : (a0.c[q0] - 1) + g.L * (a1.c[q1] - 1);
        const SubTS ts = subts[sid];
        const TypeDev& td = stypes[ts.type];
        // row index inside the member's batch row (the unclipped box for dense solves)
        const long e = (a0.u[q0] + td.off[0]) +
                       (long)td.hm[0] * ((a1.u[q1] + td.off[1]) + (long)td.hm[1] * (i2 + td.off[2]));
        if (td.dense) {
          td.Rh[(long)ts.slot * td.ld + e] = hi;
          if (td.Rl != nullptr) td.Rl[(long)ts.slot * td.ld + e] = lo;
        } else {
          td.batch[(long)ts.slot * td.nch * td.b + e] = rv;
        }
      }
    }
  }
  if (xr.on) write_partial<kBig>(acc, rr.part);
}

// ---- dense local solves: restriction and extension with arithmetic addressing
//
// With dense local solves the batch row of a subdomain is its id and every
// subdomain's box sits inside the unclipped box of its cell, so the batch
// index of a node follows from the node and cell indices alone: along an
// expanding axis the unclipped box of cell c starts at node (c - 1) n_e -
// delta, giving the box-local index i + delta - (c - 1) n_e.  The kernels
// below therefore issue all of a node's loads at once (no table look-ups in
// between); the covering cells come from covering() and the partition-of-unity
// weights from the same per-axis tables as in the generic kernels.
__device__ inline long dense_index(const Geo& g, int delta, const DenseArgs& da, const int* i,
                                   int c0, int c1) {
  const int u0 = i[0] + delta - (c0 - 1) * g.ne;
  const int u1 = g.p == 2 ? i[1] + delta - (c1 - 1) * g.ne : i[1];
  return u0 + (long)da.hm0 * (u1 + (long)da.hm1 * i[2]);
}

// Covering cells of a node: slot q = q0 + 2 q1 (q1 = 0 for one expanding
// axis) is cell (clo0 + q0, clo1 + q1) when that exists.  Out-of-range slots
// are clamped to an existing cell so that their loads stay valid and can be
// issued unconditionally; `val` masks their contributions.
template <int PX>
struct Cover {
  static constexpr int NC = PX == 1 ? 2 : 4;
  int clo0, chi0, clo1, chi1;
  __device__ Cover(const Geo& g, int delta, const int* i) {
    clo1 = chi1 = 1;
    covering(i[0] + 1, g.ne, g.L, delta, clo0, chi0);
    if (PX == 2) covering(i[1] + 1, g.ne, g.L, delta, clo1, chi1);
  }
  __device__ bool val(int q) const { return clo0 + (q & 1) <= chi0 && clo1 + (q >> 1) <= chi1; }
  __device__ int c0(int q) const { return min(clo0 + (q & 1), chi0); }
  __device__ int c1(int q) const { return min(clo1 + (q >> 1), chi1); }
};

// Bodies of the node-parallel kernels take the block index `bid` and the
// block count `nblk` of their problem (blockIdx.x / gridDim.x of a single
// problem, or the block's index and its instance's block count in a grouped
// launch).
template <int PX>
__device__ __forceinline__ void restrict_dense_body(const Geo& g, int delta,
                                                    PcgState* __restrict__ st, const XrArgs& xr,
                                                    const Red& rr, double* __restrict__ r,
                                                    const DenseArgs& da, int bid, int nblk) {
  if (st != nullptr && st->done) return;
  double alpha = 0.0;
  if (xr.on == 1) {
    const double gamma = sum_partials<kBig>(xr.gam.part, xr.gam.np);
    if (!(gamma > 0.0)) {
      if (bid == 0 && threadIdx.x == 0) {
        st->done = 2;
        st->iters = xr.k - 1;
      }
      return;
    }
    alpha = st->rho[(xr.k - 1) & 1] / gamma;
  }
  const int N0 = g.N[0], N1 = g.N[1];
  const int segs = (N0 + kBlock - 1) / kBlock;
  const long items = (long)segs * N1 * g.N[2];
  const int sub = threadIdx.x / kBlock, tx = threadIdx.x % kBlock;
  double acc = 0.0;
  // two nodes per thread and pass (items it and it + IPB), all their loads
  // issued before either is updated: the grid (node_grid_dense) fits on the
  // chip in one round
  constexpr int IPB = kBig / kBlock;
  for (long grp = bid; grp * 2 * IPB < items; grp += nblk) {
    bool ok[2];
    long kk[2];
    int ii[2][3];
    double rv[2], qv[2], pv[2], xv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long it = grp * 2 * IPB + u * IPB + sub;
      const int line = (int)(it / segs);
      const int i0 = (int)(it - (long)line * segs) * kBlock + tx;
      ok[u] = it < items && i0 < N0;
      const int i2 = g.D == 3 ? (int)fdiv((unsigned)line, g.fN1) : 0;
      ii[u][0] = i0; ii[u][1] = line - i2 * N1; ii[u][2] = i2;
      kk[u] = i0 + (long)N0 * line;
      rv[u] = qv[u] = pv[u] = xv[u] = 0.0;
      if (ok[u]) {
        rv[u] = xr.on == 2 ? xr.q[kk[u]] : r[kk[u]];
        if (xr.on == 1) {
          qv[u] = xr.q[kk[u]];
          pv[u] = xr.p[kk[u]];
          xv[u] = xr.x[kk[u]];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (!ok[u]) continue;
      const long k = kk[u];
      const int* i = ii[u];
      double rvv = rv[u];
      if (xr.on == 1) {
        rvv -= alpha * qv[u];
        xr.x[k] = xv[u] + alpha * pv[u];
        r[k] = rvv;
        acc += rvv * rvv;
      } else if (xr.on == 2) {
        xr.x[k] = 0.0;
        r[k] = rvv;
        acc += rvv * rvv;
      }
      const __bf16 hi = to_bf16(rvv);
      const __bf16 lo = to_bf16(rvv - (double)hi);
      const Cover<PX> cv(g, delta, i);
#pragma unroll
      for (int q = 0; q < Cover<PX>::NC; ++q) {
        if (!cv.val(q)) continue;
        const int c0 = cv.c0(q), c1 = cv.c1(q);
        const long at = (long)((c0 - 1) + g.L * (c1 - 1)) * da.ld + dense_index(g, delta, da, i, c0, c1);
        da.Rh[at] = hi;
        if (da.Rl != nullptr) da.Rl[at] = lo;
      }
    }
  }
  if (xr.on) write_partial_at<kBig>(acc, rr.part, bid);
}

template <int PX>
__global__ void __launch_bounds__(kBig) k_restrict_dense(Geo g, int delta, PcgState* __restrict__ st,
                                                         XrArgs xr, Red rr, double* __restrict__ r,
                                                         DenseArgs da) {
  restrict_dense_body<PX>(g, delta, st, xr, rr, r, da, blockIdx.x, gridDim.x);
}

// z = sum_c R_c^T y_c + psi_ext cf (cf from k_coarse_field when coarse != 0).
// RAS weights every local solution by the partition of unity,
// z = sum_c R_c^T D_c y_c (+ the coarse term): the restricted additive Schwarz
// extension of eq:dd-preconditioners, from the same per-axis covering tables.
// INL forms the coarse field at the node from y0 itself (cf then points to
// y0): sum_c D_c y0_c over the covering cells in slot order, the arithmetic of
// k_coarse_field.
template <int PX, int KS, bool RAS = false, bool INL = false, int NPT = 1>
__device__ __forceinline__ void extend_dense_body(const Geo& g, int delta, int coarse,
                                                  PcgState* __restrict__ st, const CheckArgs& chk,
                                                  const DenseArgs& da,
                                                  const double* __restrict__ psi,
                                                  const double* __restrict__ cf,
                                                  const double* __restrict__ r,
                                                  double* __restrict__ z, int use_dot,
                                                  const Red& dot, int bid, int nblk, int pu = 0,
                                                  const XCover* __restrict__ xc0 = nullptr,
                                                  const XCover* __restrict__ xc1 = nullptr) {
  constexpr int NC = Cover<PX>::NC;
  if (st != nullptr && st->done) return;
  if (chk.on) {
    const double rn2 = sum_partials<kBig>(chk.rr.part, chk.rr.np);
    const bool conv = rn2 <= st->tol2, last = chk.k >= chk.maxit;
    if (bid == 0 && threadIdx.x == 0) {
      st->relres = sqrt(rn2 / st->r0n2);
      if (chk.hist && chk.k < chk.hist_cap) chk.hist[chk.k] = st->relres;
      st->iters = chk.k;
      if (conv) st->done = 1;
      else if (last) st->done = 4;
    }
    if (conv || last) return;
  }
  double acc = 0.0;
  const int N0 = g.N[0], N1 = g.N[1];
  const int segs = (N0 + kBlock - 1) / kBlock;
  const long items = (long)segs * N1 * g.N[2];
  const int sub = threadIdx.x / kBlock, tx = threadIdx.x % kBlock;
  // NPT nodes per thread and pass (items it + u IPB): every load of them
  // first, then their sums
  constexpr int IPB = kBig / kBlock;
  for (long grp = bid; grp * NPT * IPB < items; grp += nblk) {
    bool okn[NPT];
    long kn[NPT];
    int in_[NPT][3];
    XCover xan[NPT];
    double yan[NPT][2], rkn[NPT];
    float zsn[NPT][NC][KS];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const long it = grp * NPT * IPB + u * IPB + sub;
      const int line = (int)(it / segs);
      const int i0 = (int)(it - (long)line * segs) * kBlock + tx;
      okn[u] = it < items && i0 < N0;
      const int i2 = g.D == 3 ? (int)fdiv((unsigned)line, g.fN1) : 0;
      in_[u][0] = i0;
      in_[u][1] = line - i2 * N1;
      in_[u][2] = i2;
      kn[u] = i0 + (long)N0 * line;
      yan[u][0] = yan[u][1] = 0.0;
      if (!okn[u]) continue;
      const Cover<PX> cv(g, delta, in_[u]);
      // (the inline coarse field with one expanding axis: the covering-table
      // entry and the two y0 values)
      if constexpr (INL && PX == 1) {
        if (coarse) {
          xan[u] = xc0[i0];
          yan[u][0] = cf[cv.c0(0) - 1];
          yan[u][1] = cf[cv.c0(1) - 1];
        }
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int c0 = cv.c0(q), c1 = cv.c1(q);
        const int sid = (c0 - 1) + g.L * (c1 - 1);
        const long at = (long)sid * da.ld + dense_index(g, delta, da, in_[u], c0, c1);
#pragma unroll
        for (int sp = 0; sp < KS; ++sp) zsn[u][q][sp] = da.Z[sp * da.zsplit + at];
      }
      rkn[u] = r[kn[u]];
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
    if (!okn[u]) continue;
    const int* i = in_[u];
    const int i0 = i[0], i2 = i[2];
    const long k = kn[u];
    const Cover<PX> cv(g, delta, i);
    const XCover& xa = xan[u];
    const double* ya = yan[u];
    float (&zs)[NC][KS] = zsn[u];
    const double rk = rkn[u];
    double ps = 0.0, zc = 0.0;
    if (coarse) {
      // cell-local table node: x dims (i + 1) mod n_e
      const int j0 = (int)((unsigned)(i0 + 1) - g.ne * fdiv((unsigned)(i0 + 1), g.fne));
      const int j1 = PX == 2 ? (int)((unsigned)(i[1] + 1) - g.ne * fdiv((unsigned)(i[1] + 1), g.fne))
                             : i[1];
      ps = psi[j0 + (long)g.P[0] * (j1 + (long)g.P[1] * i2)];
      if constexpr (INL && PX == 1) {
        // the weights of the one expanding axis (cover_weight for p = 1)
        zc = xa.w[0] * ya[0];
        if (cv.val(1)) zc = fma(xa.w[1], ya[1], zc);
      } else if constexpr (INL) {
        const XCover* xc[2] = {xc0, xc1};
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          if (!cv.val(q)) continue;
          const int c[3] = {cv.c0(q), PX == 2 ? cv.c1(q) : 0, 0};
          const int which[2] = {q & 1, q >> 1};
          zc += cover_weight(g, delta, pu, xc, c, i, which) * cf[(c[0] - 1) + g.L * (cv.c1(q) - 1)];
        }
      } else {
        zc = cf[PX == 1 ? (long)i0 : i0 + (long)N0 * i[1]];
      }
    }
    // ... then the sums, cells in slot order and splits in split order
    double zl = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (!cv.val(q)) continue;
      float zq = 0.0f;
#pragma unroll
      for (int sp = 0; sp < KS; ++sp) zq += zs[q][sp];
      if constexpr (RAS) {
        const XCover* xc[2] = {xc0, xc1};
        const int c[3] = {cv.c0(q), cv.c1(q), 0};
        const int which[2] = {q & 1, q >> 1};
        zl += cover_weight(g, delta, pu, xc, c, i, which) * (double)zq;
      } else {
        zl += (double)zq;
      }
    }
    // one rounding for the coarse term, whatever the compiler knows of `coarse`
    const double zv = coarse ? fma(ps, zc, zl) : zl;
    z[k] = zv;
    acc += rk * zv;
    }
  }
  if (use_dot) write_partial_at<kBig>(acc, dot.part, bid);
}

template <int PX, int KS, bool RAS, bool INL>
__global__ void __launch_bounds__(kBig) k_extend_dense(Geo g, int delta, int coarse,
                                                       PcgState* __restrict__ st, CheckArgs chk,
                                                       DenseArgs da, const double* __restrict__ psi,
                                                       const double* __restrict__ cf,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ z, int use_dot, Red dot,
                                                       int pu, const XCover* __restrict__ xc0,
                                                       const XCover* __restrict__ xc1) {
  extend_dense_body<PX, KS, RAS, INL>(g, delta, coarse, st, chk, da, psi, cf, r, z, use_dot, dot,
                                      blockIdx.x, gridDim.x, pu, xc0, xc1);
}

// One expanding axis: two nodes per thread on node_grid_dense's grid, at most
// 64 VGPRs so that two 1024-thread workgroups fit on a CU (one round).
template <int KS, bool RAS, bool INL>
__global__ void __launch_bounds__(kBig) __attribute__((amdgpu_waves_per_eu(8)))
k_extend_dense_p1(Geo g, int delta, int coarse,
                                                       PcgState* __restrict__ st, CheckArgs chk,
                                                       DenseArgs da, const double* __restrict__ psi,
                                                       const double* __restrict__ cf,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ z, int use_dot, Red dot,
                                                       int pu, const XCover* __restrict__ xc0,
                                                       const XCover* __restrict__ xc1) {
  extend_dense_body<1, KS, RAS, INL, 2>(g, delta, coarse, st, chk, da, psi, cf, r, z, use_dot, dot,
                                      blockIdx.x, gridDim.x, pu, xc0, xc1);
}

DenseArgs dense_args(const ddeig_problem* P) {
  const DenseHost& H = P->dh;
  return DenseArgs{H.Rh, H.Rl, H.Z, (long)H.mp * H.ld, H.ld, P->ksplit, H.box.m[0], H.box.m[1]};
}

// Workgroups of the node-parallel kernels: four row segments per workgroup,
// at most kMaxRed workgroups (partial-sum capacity).
int node_grid(const Geo& g) {
  const long segs = (g.N[0] + kBlock - 1) / kBlock;
  const long items = segs * g.N[1] * g.N[2];
  const long groups = (items + kBig / kBlock - 1) / (kBig / kBlock);
  return (int)std::max<long>(1, std::min<long>(groups, kMaxRed));
}

// The dense restriction and (one expanding axis, additive) extension take two
// items per thread and pass; a batch uses the same count per instance, so its
// partial sums match the single problem's bit for bit.
int node_grid_dense(const Geo& g) {
  const long segs = (g.N[0] + kBlock - 1) / kBlock;
  const long items = segs * g.N[1] * g.N[2];
  const long groups = (items + 2 * (kBig / kBlock) - 1) / (2 * (kBig / kBlock));
  return (int)std::max<long>(1, std::min<long>(groups, kMaxRed));
}

void launch_restrict(const ddeig_problem* P, double* r, PcgState* st, const XrArgs& xr, Red* rr,
                     hipStream_t s) {
  const int blocks = P->opt.local_prec >= 2 ? node_grid_dense(P->g) : node_grid(P->g);
  const Red none{nullptr, 0, nullptr};
  if (xr.on) rr->np = blocks;
  if (P->opt.local_prec >= 2) {
    if (P->g.p == 1)
      hipLaunchKernelGGL(k_restrict_dense<1>, dim3(blocks), dim3(kBig), 0, s, P->g, P->delta, st,
                         xr, xr.on ? *rr : none, r, dense_args(P));
    else
      hipLaunchKernelGGL(k_restrict_dense<2>, dim3(blocks), dim3(kBig), 0, s, P->g, P->delta, st,
                         xr, xr.on ? *rr : none, r, dense_args(P));
  } else
    hipLaunchKernelGGL(k_restrict, dim3(blocks), dim3(kBig), 0, s, P->g, (int)P->types.size(), st,
                       xr, xr.on ? *rr : none, r, P->dTypes, P->dSubTS, P->dXC[0], P->dXC[1]);
}

__global__ void __launch_bounds__(kBlock) k_coarse_rhs(Geo g, const PcgState* __restrict__ st,
                                                       const double* __restrict__ r,
                                                       const TypeDev* __restrict__ types,
                                                       const SubDev* __restrict__ subs,
                                                       double* __restrict__ crhs) {
  coarse_rhs_body(g, st, r, types, subs, crhs, blockIdx.x);
}

void launch_coarse_rhs(const ddeig_problem* P, const double* r, const PcgState* st,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_rhs, dim3(P->nsub), dim3(kBlock), 0, s, P->g, st, r, P->dTypes,
                     P->dSubs, P->crhs);
}

// phi of every class from its first member's box: D_c(k) psi_ext(k).
__global__ void k_coarse_phi(Geo g, int delta, int pu, const TypeDev* __restrict__ types,
                             const SubDev* __restrict__ subs, const int* __restrict__ first,
                             const XCover* __restrict__ xc0, const XCover* __restrict__ xc1,
                             const double* __restrict__ psi, double* const* __restrict__ phis) {
  const int t = blockIdx.y;
  const TypeDev td = types[t];
  const SubDev sd = subs[first[t]];
  const XCover* xc[2] = {xc0, xc1};
  const int m0 = td.m[0], m1 = td.m[1];
  const int mtot = m0 * m1 * td.m[2];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < mtot; e += gridDim.x * blockDim.x) {
    const int line = e / m0, u0 = e - line * m0;
    const int u2 = line / m1, u1 = line - u2 * m1;
    const int i[3] = {sd.o[0] + u0, sd.o[1] + u1, sd.o[2] + u2};
    int which[2] = {0, 0};
    for (int a = 0; a < g.p; ++a) which[a] = xc[a][i[a]].c[0] == sd.c[a] ? 0 : 1;
    phis[t][e] = cover_weight(g, delta, pu, xc, sd.c, i, which) *
                 psi[table_node(g, i[0], i[1], i[2])];
  }
}

void launch_coarse_phi(const ddeig_problem* P, hipStream_t s) {
  const int nt = (int)P->types.size();
  hipLaunchKernelGGL(k_coarse_phi, dim3(64, nt), dim3(kBlock), 0, s, P->g, P->delta, P->opt.pu,
                     P->dTypes, P->dSubs, P->dFirst, P->dXC[0], P->dXC[1], P->psi, P->dPhis);
}

__global__ void k_coarse_solve(int N, const PcgState* __restrict__ st,
                               const double* __restrict__ A0inv, const double* __restrict__ c,
                               double* __restrict__ y) {
  coarse_solve_body(N, st, A0inv, c, y, blockIdx.x);
}

void launch_coarse_solve(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  const int rows_per_block = kBlock / 64;
  hipLaunchKernelGGL(k_coarse_solve, dim3((P->nsub + rows_per_block - 1) / rows_per_block),
                     dim3(kBlock), 0, s, P->nsub, st, P->A0inv, P->crhs, P->cy);
}

// The coarse correction R_0^T y0 at a node is psi_ext(node) times
// sum_c D_c(node) y0_c over the covering cells c, and both the covering cells
// and the weights depend only on the node's expanding indices.  This kernel
// forms that sum once per expanding-index point (i0, or (i0, i1) for two
// expanding axes), cells in slot order, so the extension reads one value.
template <int PX>
__device__ __forceinline__ void coarse_field_body(const Geo& g, int delta, int pu,
                                                  const PcgState* __restrict__ st,
                                                  const XCover* __restrict__ xc0,
                                                  const XCover* __restrict__ xc1,
                                                  const double* __restrict__ y0,
                                                  double* __restrict__ cf, int bid, int nblk) {
  if (st != nullptr && st->done) return;
  const XCover* xc[2] = {xc0, xc1};
  const long npts = PX == 1 ? (long)g.N[0] : (long)g.N[0] * g.N[1];
  for (long idx = bid * (long)blockDim.x + threadIdx.x; idx < npts;
       idx += (long)nblk * blockDim.x) {
    const int i[3] = {(int)(idx % g.N[0]), PX == 2 ? (int)(idx / g.N[0]) : 0, 0};
    const Cover<PX> cv(g, delta, i);
    double zc = 0.0;
#pragma unroll
    for (int q = 0; q < Cover<PX>::NC; ++q) {
      if (!cv.val(q)) continue;
      const int c[3] = {cv.c0(q), PX == 2 ? cv.c1(q) : 0, 0};
      const int which[2] = {q & 1, q >> 1};
      zc += cover_weight(g, delta, pu, xc, c, i, which) * y0[(c[0] - 1) + g.L * (cv.c1(q) - 1)];
    }
    cf[idx] = zc;
  }
}

template <int PX>
__global__ void k_coarse_field(Geo g, int delta, int pu, const PcgState* __restrict__ st,
                               const XCover* __restrict__ xc0, const XCover* __restrict__ xc1,
                               const double* __restrict__ y0, double* __restrict__ cf) {
  coarse_field_body<PX>(g, delta, pu, st, xc0, xc1, y0, cf, blockIdx.x, gridDim.x);
}

void launch_coarse_field(const ddeig_problem* P, const PcgState* st, hipStream_t s) {
  const long npts = P->g.p == 1 ? (long)P->g.N[0] : (long)P->g.N[0] * P->g.N[1];
  const int blocks = (int)std::min<long>((npts + kBlock - 1) / kBlock, 4096);
  if (P->g.p == 1)
    hipLaunchKernelGGL(k_coarse_field<1>, dim3(blocks), dim3(kBlock), 0, s, P->g, P->delta,
                       P->opt.pu, st, P->dXC[0], P->dXC[1], P->cy, P->cfield);
  else
    hipLaunchKernelGGL(k_coarse_field<2>, dim3(blocks), dim3(kBlock), 0, s, P->g, P->delta,
                       P->opt.pu, st, P->dXC[0], P->dXC[1], P->cy, P->cfield);
}

// z = sum_c R_c^T y_c (+ R_0^T y0), partials of r.z.  Work items are row
// segments of kBlock x1 positions, four per workgroup of kBig threads (as in
// the restriction); the covering cells of a node come from the per-axis
// tables and are summed in a fixed order.
// With chk.on the kernel first applies the stopping test of PCG iteration k,
// ||r_k|| <= rtol ||r_0|| (§4.1), records the history and, once CG stops,
// does nothing else (every later kernel of the iteration sees `done`).
__global__ void __launch_bounds__(kBig) k_extend(Geo g, int delta, int pu, int coarse, int ras,
                                                   int ntypes, PcgState* __restrict__ st,
                                                   CheckArgs chk,
                                                   const TypeDev* __restrict__ types,
                                                   const SubTS* __restrict__ subts,
                                                   const XCover* __restrict__ xc0,
                                                   const XCover* __restrict__ xc1,
                                                   const double* __restrict__ psi,
                                                   const double* __restrict__ y0,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ z, int use_dot,
                                                   Red dot) {
  __shared__ TypeDev stypes[kMaxTypes];
  if (st != nullptr && st->done) return;
  if (chk.on) {
    const double rn2 = sum_partials<kBig>(chk.rr.part, chk.rr.np);
    const bool conv = rn2 <= st->tol2, last = chk.k >= chk.maxit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->relres = sqrt(rn2 / st->r0n2);
      if (chk.hist && chk.k < chk.hist_cap) chk.hist[chk.k] = st->relres;
      st->iters = chk.k;
      if (conv) st->done = 1;
      else if (last) st->done = 4;
    }
    if (conv || last) return;
  }
  if (threadIdx.x < ntypes) stypes[threadIdx.x] = types[threadIdx.x];
  __syncthreads();
  const XCover* xc[2] = {xc0, xc1};
  double acc = 0.0;
  const int N0 = g.N[0], N1 = g.N[1];
  const int segs = (N0 + kBlock - 1) / kBlock;
  const long items = (long)segs * N1 * g.N[2];
  const int sub = threadIdx.x / kBlock, tx = threadIdx.x % kBlock;
  for (long grp = blockIdx.x; grp * (kBig / kBlock) < items; grp += gridDim.x) {
    const long it = grp * (kBig / kBlock) + sub;
    if (it >= items) continue;
    const int line = (int)(it / segs);
    const int i0 = (int)(it - (long)line * segs) * kBlock + tx;
    if (i0 >= N0) continue;
    const int i2 = g.D == 3 ? (int)fdiv((unsigned)line, g.fN1) : 0;
    const int i[3] = {i0, line - i2 * N1, i2};
    const long k = i0 + (long)N0 * line;
    const XCover a0 = xc0[i0];
    XCover a1;
    a1.c[0] = 1; a1.c[1] = 0; a1.u[0] = i[1]; a1.u[1] = 0; a1.w[0] = 1.0; a1.w[1] = 0.0;
    if (g.p == 2) a1 = xc1[i[1]];
    double zl = 0.0, zc = 0.0;
    for (int q1 = 0; q1 < 2; ++q1) {
      if (a1.c[q1] == 0) continue;
      for (int q0 = 0; q0 < 2; ++q0) {
        if (a0.c[q0] == 0) continue;
        const int c[3] = {a0.c[q0], g.p == 2 ? a1.c[q1] : 0, 0};
        const int sid = sub_index(g, c);
        const SubTS ts = subts[sid];
        const TypeDev& td = stypes[ts.type];
        const int u1 = g.p == 2 ? a1.u[q1] : i[1];
        const long e = (a0.u[q0] + td.off[0]) +
                       (long)td.hm[0] * ((u1 + td.off[1]) + (long)td.hm[1] * (i2 + td.off[2]));
        double zi;
        if (td.dense) {
          const float* zp = td.Z + (long)ts.slot * td.ld + e;
          float zs = 0.0f;
          for (int sp = 0; sp < td.ksplit; ++sp) zs += zp[sp * td.zsplit];
          zi = (double)zs;
        } else {
          zi = td.batch[(long)ts.slot * td.nch * td.b + e];
        }
        const int which[2] = {q0, q1};
        const double wc = (coarse || ras) ? cover_weight(g, delta, pu, xc, c, i, which) : 1.0;
        zl += ras ? wc * zi : zi;
        if (coarse) zc += wc * y0[sid];
      }
    }
    double zv = zl;
    if (coarse) zv += psi[table_node(g, i[0], i[1], i[2])] * zc;
    z[k] = zv;
    acc += r[k] * zv;
  }
  if (use_dot) write_partial<kBig>(acc, dot.part);
}

template <bool RAS, bool INL>
static auto dense_extend_kernel(int p, int ks) {
  if (p == 1 && !RAS)  // (the RAS weights would spill at 64 VGPRs)
    return ks == 1 ? k_extend_dense_p1<1, RAS, INL>
                   : (ks == 2 ? k_extend_dense_p1<2, RAS, INL> : k_extend_dense_p1<3, RAS, INL>);
  if (p == 1)
    return ks == 1 ? k_extend_dense<1, 1, RAS, INL>
                   : (ks == 2 ? k_extend_dense<1, 2, RAS, INL> : k_extend_dense<1, 3, RAS, INL>);
  return ks == 1 ? k_extend_dense<2, 1, RAS, INL>
                 : (ks == 2 ? k_extend_dense<2, 2, RAS, INL> : k_extend_dense<2, 3, RAS, INL>);
}

// inline_field: the coarse field is formed in the extension from y0 (P->cy)
// instead of read from k_coarse_field's output (dense local solves only).
void launch_extend(const ddeig_problem* P, const double* r, double* z, int coarse, Red* dot,
                   PcgState* st, const CheckArgs& chk, hipStream_t s, int ras, int inline_field) {
  const int blocks = P->opt.local_prec >= 2 && P->g.p == 1 && !ras ? node_grid_dense(P->g)
                                                                   : node_grid(P->g);
  const Red none{nullptr, 0, nullptr};
  if (dot) dot->np = blocks;
  if (P->opt.local_prec >= 2) {
    // the K split is 1..3 by construction (assemble)
    const bool inl = coarse && inline_field;
    auto kern = ras ? (inl ? dense_extend_kernel<true, true>(P->g.p, P->ksplit)
                           : dense_extend_kernel<true, false>(P->g.p, P->ksplit))
                    : (inl ? dense_extend_kernel<false, true>(P->g.p, P->ksplit)
                           : dense_extend_kernel<false, false>(P->g.p, P->ksplit));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBig), 0, s, P->g, P->delta, coarse, st, chk,
                       dense_args(P), P->psi, inl ? P->cy : P->cfield, r, z, dot ? 1 : 0,
                       dot ? *dot : none, P->opt.pu, P->dXC[0], P->dXC[1]);
    return;
  }
  hipLaunchKernelGGL(k_extend, dim3(blocks), dim3(kBig), 0, s, P->g, P->delta, P->opt.pu,
                     coarse, ras, (int)P->types.size(), st, chk, P->dTypes, P->dSubTS, P->dXC[0],
                     P->dXC[1],
                     P->psi, P->cy, r, z,
                     dot ? 1 : 0, dot ? *dot : none);
}

// The coarse correction alone, z = R_0^T y0 = psi_ext * cf at every node
// (cf from k_coarse_field), with the partials of r.z when use_dot: the
// correction step of eq:two-level-stationary-ras-mult-cc.
__global__ void __launch_bounds__(kBlock) k_coarse_extend(Geo g, const PcgState* __restrict__ st,
                                                          const double* __restrict__ psi,
                                                          const double* __restrict__ cf,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ z, int use_dot,
                                                          Red dot) {
  if (st != nullptr && st->done) return;
  double acc = 0.0;
  for (long k = blockIdx.x * (long)kBlock + threadIdx.x; k < g.n; k += (long)gridDim.x * kBlock) {
    int i0, i1, i2;
    unflatten(g, k, i0, i1, i2);
    const double v = psi[table_node(g, i0, i1, i2)] * cf[g.p == 1 ? (long)i0 : i0 + (long)g.N[0] * i1];
    z[k] = v;
    acc += r[k] * v;
  }
  if (use_dot) write_partial(acc, dot.part);
}

void launch_coarse_extend(const ddeig_problem* P, const double* r, double* z, Red* dot,
                          const PcgState* st, hipStream_t s) {
  const int blocks = (int)std::max<long>(1, std::min<long>((P->g.n + kBlock - 1) / kBlock, kMaxRed));
  const Red none{nullptr, 0, nullptr};
  if (dot) dot->np = blocks;
  hipLaunchKernelGGL(k_coarse_extend, dim3(blocks), dim3(kBlock), 0, s, P->g, st, P->psi,
                     P->cfield, r, z, dot ? 1 : 0, dot ? *dot : none);
}

// phi_c(k) = D_c(k) psi_ext(k) on box c, 0 elsewhere (column c of R_0^T).
__device__ inline double coarse_phi(const Geo& g, int delta, int pu, const SubDev& sd,
                                    const TypeDev& td, const double* psi, const int* i) {
  for (int a = 0; a < g.D; ++a)
    if (i[a] < sd.o[a] || i[a] >= sd.o[a] + td.m[a]) return 0.0;
  return pu_weight(g, delta, pu, sd.c, i) * psi[table_node(g, i[0], i[1], i[2])];
}

// A0[c][d] = phi_d^T A_sigma phi_c for neighbouring cells (one workgroup per pair).
__global__ void __launch_bounds__(kBlock) k_coarse_matrix(Geo g, int delta, int pu,
                                                          const double* __restrict__ T,
                                                          const TypeDev* __restrict__ types,
                                                          const SubDev* __restrict__ subs,
                                                          const double* __restrict__ psi,
                                                          double* __restrict__ A0) {
  const int N = gridDim.x;
  const int cid = blockIdx.x;
  const int nb = blockIdx.y;  // neighbour offset in {-1,0,1}^p
  const SubDev sc = subs[cid];
  int dc[2] = {nb % 3 - 1, nb / 3 - 1};
  int cd[3] = {sc.c[0] + dc[0], g.p == 2 ? sc.c[1] + dc[1] : 0, 0};
  if (g.p == 1 && dc[1] != -1) return;  // only nb in {0,1,2} for p = 1
  for (int a = 0; a < g.p; ++a)
    if (cd[a] < 1 || cd[a] > g.L) return;
  const int did = sub_index(g, cd);
  const SubDev sdd = subs[did];
  const TypeDev tc = types[sc.type];
  const TypeDev tdd = types[sdd.type];
  const long mtot = (long)tdd.m[0] * tdd.m[1] * tdd.m[2];
  double acc = 0.0;
  for (long e = threadIdx.x; e < mtot; e += blockDim.x) {
    const int i[3] = {sdd.o[0] + (int)(e % tdd.m[0]), sdd.o[1] + (int)((e / tdd.m[0]) % tdd.m[1]),
                      sdd.o[2] + (int)(e / ((long)tdd.m[0] * tdd.m[1]))};
    const double phid = coarse_phi(g, delta, pu, sdd, tdd, psi, i);
    const long tn = table_node(g, i[0], i[1], i[2]);
    double aphi = 0.0;
    for (int t = 0; t < g.ntaps; ++t) {
      int d[3];
      tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
      const int j[3] = {i[0] + d[0], i[1] + d[1], g.D == 3 ? i[2] + d[2] : 0};
      bool in = true;
      for (int a = 0; a < g.D; ++a) in = in && j[a] >= 0 && j[a] < g.N[a];
      if (!in) continue;
      aphi += T[t * g.tsize + tn] * coarse_phi(g, delta, pu, sc, tc, psi, j);
    }
    acc += phid * aphi;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) A0[(long)cid * N + did] = s;
}

__global__ void k_symmetrise(double* A, int N) {
  const long nn = (long)N * N;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < nn;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / N), j = (int)(idx % N);
    if (j > i) {
      const double v = 0.5 * (A[idx] + A[(long)j * N + i]);
      A[idx] = v;
      A[(long)j * N + i] = v;
    }
  }
}

void launch_symmetrise(double* A, int N, hipStream_t s) {
  const long nn = (long)N * N;
  const int blocks = (int)std::min<long>((nn + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_symmetrise, dim3(blocks), dim3(kBlock), 0, s, A, N);
}

void build_coarse_matrix(ddeig_problem* P, double* A0, hipStream_t s) {
  const int N = P->nsub;
  check_hip(hipMemsetAsync(A0, 0, sizeof(double) * (size_t)N * N, s), "memset A0");
  const int nnb = P->g.p == 1 ? 3 : 9;
  // for p = 1 the neighbour offsets are encoded as nb = 0,1,2 with dc[1] = -1
  hipLaunchKernelGGL(k_coarse_matrix, dim3(N, nnb), dim3(kBlock), 0, s, P->g, P->delta,
                     P->opt.pu, P->tabAs, P->dTypes, P->dSubs, P->psi, A0);
  launch_symmetrise(A0, N, s);
}

int coarse_field_grid(const Geo& g) {
  const long npts = g.p == 1 ? (long)g.N[0] : (long)g.N[0] * g.N[1];
  return (int)std::max<long>(1, std::min<long>((npts + kBlock - 1) / kBlock, 4096));
}

// Grouped kernels of PCG iteration k over the instances of a batch (2-D,
// one expanding axis, dense local solves): block b runs block map[b].y of
// instance map[b].x with that instance's operands, CG state and partials.
__global__ void __launch_bounds__(kBig) k_b_restrict(const InstDev* __restrict__ I,
                                                     const int2* __restrict__ map, int k) {
  const int2 m = map[blockIdx.x];
  const InstDev& d = I[m.x];
  const XrArgs xr{1, k, d.gam, d.x, d.pp[k & 1], d.q};
  restrict_dense_body<1>(d.g, d.delta, d.st, xr, d.rr, d.r, d.da, m.y, d.nb_node);
}

// PCG from x_0 = 0 with b = w (the batch's inverse iteration): r_0 = w,
// x_0 = 0, the partials of ||r_0||^2 and the restriction of r_0, for the
// instances with act[j] != 0 (their CG state is set afterwards).
__global__ void __launch_bounds__(kBig) k_b_restrict_start(const InstDev* __restrict__ I,
                                                           const int2* __restrict__ map,
                                                           const int* __restrict__ act) {
  const int2 m = map[blockIdx.x];
  if (!act[m.x]) return;
  const InstDev& d = I[m.x];
  const XrArgs xr{2, 0, d.rr, d.x, nullptr, d.w};
  restrict_dense_body<1>(d.g, d.delta, nullptr, xr, d.rr, d.r, d.da, m.y, d.nb_node);
}

__global__ void k_b_pcg_init(const InstDev* __restrict__ I, const int* __restrict__ act,
                             double rtol) {
  const int j = blockIdx.x;
  if (!act[j]) return;
  pcg_init_body(I[j].st, rtol, I[j].rr, I[j].hist, 0.0);
}

// Inverse-iteration normalisation (as k_ipm_normalise) of every instance with
// act[j] != 0: x_new = sign(1^T M u) u / sqrt(u^T M u) into xo, and the
// partials of ||x_new - x||_M^2 = (x_new - x)^T (scale Mu - b) (Mu in z, b in w).
__global__ void __launch_bounds__(kBig) k_b_normalise(const InstDev* __restrict__ I,
                                                      const int2* __restrict__ map,
                                                      const int* __restrict__ act) {
  const int2 m = map[blockIdx.x];
  if (!act[m.x]) return;
  const InstDev& d = I[m.x];
  const double ssum = sum_partials<kBig>(d.nm_sum.part, d.nm_sum.np);
  const double uu = sum_partials<kBig>(d.nm_uMu.part, d.nm_uMu.np);
  const double sc = (ssum < 0.0 ? -1.0 : 1.0) / sqrt(uu);
  const long n = d.g.n;
  double acc = 0.0;
  for (long i = m.y * (long)kBig + threadIdx.x; i < n; i += (long)d.nb_node * kBig) {
    const double xn = sc * d.x[i];
    const double dd = xn - d.xo[i];
    acc += dd * (sc * d.z[i] - d.w[i]);
    d.xo[i] = xn;
  }
  write_partial_at<kBig>(acc, d.nm_dx.part, m.y);
}

// res[2 j] = ||x_new - x||_M^2, res[2 j + 1] = x_new^T A_sigma x_new (act[j] != 0).
__global__ void k_b_finish_norm(const InstDev* __restrict__ I, const int* __restrict__ act,
                                double* __restrict__ res) {
  const int j = blockIdx.x;
  if (!act[j]) return;
  const double dx = sum_partials(I[j].nm_dx.part, I[j].nm_dx.np);
  const double xq = sum_partials(I[j].nm_xq.part, I[j].nm_xq.np);
  if (threadIdx.x == 0) {
    res[2 * j] = dx;
    res[2 * j + 1] = xq;
  }
}

template <int KS>
// Two nodes per thread on node_grid_dense's grid, as the single problem's
// extension; check = 0 at the start of CG (z_0 and the partials of r_0.z_0 only).
__global__ void __launch_bounds__(kBig) __attribute__((amdgpu_waves_per_eu(8)))
k_b_extend(const InstDev* __restrict__ I, const int2* __restrict__ map, int k, int maxit,
           int check) {
  const int2 m = map[blockIdx.x];
  const InstDev& d = I[m.x];
  const CheckArgs chk{check, k, maxit, d.hist_cap, d.rr, d.hist};
  extend_dense_body<1, KS, false, false, 2>(d.g, d.delta, 1, d.st, chk, d.da, d.psi, d.cf, d.r,
                                            d.z, 1, d.rz, m.y, d.nb_node);
}

// The coarse right-hand side (R_0 r)_i of one subdomain by one wave, in the
// order of coarse_rhs_body's workgroup of kBlock threads: lane l keeps the
// partial sums of that workgroup's threads l + 64 w (w < kBlock / 64), takes
// each through the same shuffle tree and adds the wave sums to 0 in w order,
// so the two give identical bits.  A batch has thousands of subdomains; a
// wave each needs no workgroup barrier and holds fewer of the CUs that the
// GEMM on the other stream is using (64 instances: 57 -> 75 us for this
// kernel, 91 -> 78 us for the overlapping GEMM, 456 -> 446 ms per solve).
__device__ __forceinline__ void coarse_rhs_wave(const Geo& g, const PcgState* __restrict__ st,
                                                const double* __restrict__ r,
                                                const TypeDev* __restrict__ types,
                                                const SubDev* __restrict__ subs,
                                                double* __restrict__ crhs, int sid) {
  constexpr int U = 8, NW = kBlock / 64;
  if (st != nullptr && st->done) return;
  const int lane = threadIdx.x & 63;
  const SubDev sd = subs[sid];
  const TypeDev td = types[sd.type];
  const int m0 = td.m[0], m1 = td.m[1];
  const int mtot = m0 * m1 * td.m[2];
  double acc[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) acc[w] = 0.0;
  for (int base = 0; base < mtot; base += U * kBlock) {
    // every load of the pass first (the steps past the subdomain's end add
    // only zeros and are skipped), then the sums in the workgroup's order
    double ph[U][NW], rv[U][NW];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int e = base + q * kBlock + 64 * w + lane;
        ph[q][w] = rv[q][w] = 0.0;
        if (base + q * kBlock < mtot && e < mtot) {
          const int line = (int)fdiv((unsigned)e, td.fm0);
          const int u0 = e - line * m0;
          const int u2 = line / m1, u1 = line - u2 * m1;
          ph[q][w] = td.phi[e];
          rv[q][w] = r[(sd.o[0] + u0) +
                       (long)g.N[0] * ((sd.o[1] + u1) + (long)g.N[1] * (sd.o[2] + u2))];
        }
      }
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < NW; ++w) acc[w] += ph[q][w] * rv[q][w];
  }
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    double v = acc[w];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    t += v;
  }
  if (lane == 0) crhs[sid] = t;
}

// One wave per (instance, subdomain) entry of the map.
__global__ void __launch_bounds__(kBlock) k_b_coarse_rhs(const InstDev* __restrict__ I,
                                                         const int2* __restrict__ map, int nmap) {
  const int b = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
  if (b >= nmap) return;
  const int2 m = map[b];
  const InstDev& d = I[m.x];
  coarse_rhs_wave(d.g, d.st, d.r, d.types, d.subs, d.crhs, m.y);
}

__global__ void k_b_coarse_solve(const InstDev* __restrict__ I, const int2* __restrict__ map) {
  const int2 m = map[blockIdx.x];
  const InstDev& d = I[m.x];
  coarse_solve_body(d.nsub, d.st, d.A0inv, d.crhs, d.cy, m.y);
}

__global__ void k_b_coarse_field(const InstDev* __restrict__ I, const int2* __restrict__ map) {
  const int2 m = map[blockIdx.x];
  const InstDev& d = I[m.x];
  coarse_field_body<1>(d.g, d.delta, d.pu, d.st, d.xc0, nullptr, d.cy, d.cf, m.y, d.nb_cf);
}

// Copies every instance's CG state into out[] (the host reads them with one
// copy); with mark_done the states are first set to finished (5), so that an
// instance whose solve is not started stays idle in the grouped kernels.
__global__ void k_b_states(const InstDev* __restrict__ I, int n, PcgState* __restrict__ out,
                           int mark_done) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    PcgState* st = I[j].st;
    if (mark_done) st->done = 5;
    out[j] = *st;
  }
}

void launch_b_restrict(const InstDev* I, const BlockMap& bm, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_b_restrict, dim3(bm.nblocks), dim3(kBig), 0, s, I, bm.map, k);
}

void launch_b_extend(const InstDev* I, const BlockMap& bm, int k, int maxit, int ksplit,
                     hipStream_t s, int check) {
  auto kern = ksplit == 1 ? k_b_extend<1> : (ksplit == 2 ? k_b_extend<2> : k_b_extend<3>);
  hipLaunchKernelGGL(kern, dim3(bm.nblocks), dim3(kBig), 0, s, I, bm.map, k, maxit, check);
}

void launch_b_restrict_start(const InstDev* I, const BlockMap& bm, const int* act, hipStream_t s) {
  hipLaunchKernelGGL(k_b_restrict_start, dim3(bm.nblocks), dim3(kBig), 0, s, I, bm.map, act);
}

void launch_b_pcg_init(const InstDev* I, int n, const int* act, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(k_b_pcg_init, dim3(n), dim3(kBlock), 0, s, I, act, rtol);
}

void launch_b_normalise(const InstDev* I, const BlockMap& bm, const int* act, hipStream_t s) {
  hipLaunchKernelGGL(k_b_normalise, dim3(bm.nblocks), dim3(kBig), 0, s, I, bm.map, act);
}

void launch_b_finish_norm(const InstDev* I, int n, const int* act, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_b_finish_norm, dim3(n), dim3(kBlock), 0, s, I, act, res);
}

void launch_b_coarse_rhs(const InstDev* I, const BlockMap& bm, hipStream_t s) {
  constexpr int wpb = kBlock / 64;
  hipLaunchKernelGGL(k_b_coarse_rhs, dim3((bm.nblocks + wpb - 1) / wpb), dim3(kBlock), 0, s, I,
                     bm.map, bm.nblocks);
}

void launch_b_coarse_solve(const InstDev* I, const BlockMap& bm, hipStream_t s) {
  hipLaunchKernelGGL(k_b_coarse_solve, dim3(bm.nblocks), dim3(kBlock), 0, s, I, bm.map);
}

void launch_b_coarse_field(const InstDev* I, const BlockMap& bm, hipStream_t s) {
  hipLaunchKernelGGL(k_b_coarse_field, dim3(bm.nblocks), dim3(kBlock), 0, s, I, bm.map);
}

void launch_b_states(const InstDev* I, int n, PcgState* out, int mark_done, hipStream_t s) {
  hipLaunchKernelGGL(k_b_states, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, I, n, out,
                     mark_done);
}

}  // namespace ddeig

// Period-cell operator tables and the matrix-free Q1 stencil operator.
//
// §2 (eq:discrete-weak-form): A = K + M_V, B = M from Q1 elements on the
// translated unit-cell mesh.  By assumption A1 (V of period 1 in x) and the
// uniform mesh, the 3^d stencil coefficients of a node depend only on its
// cell-local x position (node index mod n_e) and on its fixed-direction
// indices, so one table over the period cell describes the operator on any
// Omega_L.  The potential term uses the tensor 2-point Gauss-Legendre rule per
// element, V evaluated at cell-local x.
#include "k_common.h"

namespace ddeig {

// 1-D assembled linear-element stiffness and mass at a node: centre and off-diagonal.
__device__ inline double k1(int d, double h) { return d == 0 ? 2.0 / h : -1.0 / h; }
__device__ inline double m1(int d, double h) { return d == 0 ? 4.0 * h / 6.0 : h / 6.0; }

// Potential-weighted mass entry of one (table node, tap): the element
// integrals of W N_j N_{j+d} over the elements shared by the node and its
// neighbour, tensor 2-point Gauss-Legendre rule, W at cell-local x.  The
// loops visit the elements in increasing index and the quadrature points in a
// fixed order, and the shape-function product is formed symmetrically, so
// the entries of (j, j+d) and (j+d, j) come out bit-identical.
__device__ inline double weight_entry(const Geo& g, const VSpec& v, int t, long tn) {
  const double xi_lo = 0.5 * (1.0 - 0.57735026918962576450914878050196);
  const double xi_hi = 0.5 * (1.0 + 0.57735026918962576450914878050196);
  int d[3];
  tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
  int j[3];
  j[0] = (int)(tn % g.P[0]);
  j[1] = (int)((tn / g.P[0]) % g.P[1]);
  j[2] = (int)(tn / ((long)g.P[0] * g.P[1]));
  const double h = g.h;
  // elements e_a in {gnode-1, gnode} (d=0), {gnode} (d=+1), {gnode-1} (d=-1)
  int gnode[3], ecount[3], efirst[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= g.D) {
      gnode[a] = 0; ecount[a] = 1; efirst[a] = 0;
      continue;
    }
    gnode[a] = g.isx[a] ? j[a] : j[a] + 1;
    if (d[a] == 0) { efirst[a] = gnode[a] - 1; ecount[a] = 2; }
    else if (d[a] == 1) { efirst[a] = gnode[a]; ecount[a] = 1; }
    else { efirst[a] = gnode[a] - 1; ecount[a] = 1; }
  }
  double mv = 0.0;
  for (int e2 = 0; e2 < ecount[2]; ++e2)
    for (int e1 = 0; e1 < ecount[1]; ++e1)
      for (int e0 = 0; e0 < ecount[0]; ++e0) {
        const int ee[3] = {efirst[0] + e0, efirst[1] + e1, efirst[2] + e2};
        double lo[3];
        int lj[3], ln[3];
        for (int a = 0; a < g.D; ++a) {
          const int ea = ee[a];
          lo[a] = g.isx[a] ? (double)(((ea % g.ne) + g.ne) % g.ne) * h : (double)ea * h;
          lj[a] = gnode[a] - ea;
          ln[a] = gnode[a] + d[a] - ea;
        }
        double sum = 0.0;
        const int nq = 1 << g.D;
        // QUAD_TABLE: the element's place in the period cell (x cell-local)
        long tab0 = 0;
        if (v.kind == DDEIG_V_QUAD_TABLE) {
          long stride = nq;
          for (int a = 0; a < g.D; ++a) {
            const int nel = g.isx[a] ? g.ne : g.nel[a];
            const int ea = g.isx[a] ? ((ee[a] % g.ne) + g.ne) % g.ne : ee[a];
            tab0 += stride * ea;
            stride *= nel;
          }
        }
        for (int qi = 0; qi < nq; ++qi) {
          double z[3] = {0.0, 0.0, 0.0};
          double shape = 1.0;
          for (int a = 0; a < g.D; ++a) {
            const double xi = ((qi >> a) & 1) ? xi_hi : xi_lo;
            z[a] = lo[a] + h * xi;
            const double Nj = lj[a] ? xi : 1.0 - xi;
            const double Nn = ln[a] ? xi : 1.0 - xi;
            shape *= Nj * Nn;
          }
          const double vq = v.kind == DDEIG_V_QUAD_TABLE ? v.table[tab0 + qi] : eval_V(v, z);
          sum += vq * shape;
        }
        double wvol = 1.0;
        for (int a = 0; a < g.D; ++a) wvol *= 0.5 * h;
        mv += wvol * sum;
      }
  return mv;
}

// Table entries of one (table node, tap): K, M and A = K + M_V.
__global__ void k_build_tables(Geo g, const VSpec* __restrict__ vs, double* __restrict__ tK,
                               double* __restrict__ tM, double* __restrict__ tA) {
  const long total = g.tsize * g.ntaps;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int t = (int)(idx / g.tsize);
    const long tn = idx % g.tsize;
    int d[3];
    tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
    const double h = g.h;
    // constant-coefficient parts
    double kk = 0.0, mm = 1.0;
    for (int a = 0; a < g.D; ++a) mm *= m1(d[a], h);
    for (int dir = 0; dir < g.D; ++dir) {
      double term = 1.0;
      for (int a = 0; a < g.D; ++a) term *= (a == dir) ? k1(d[a], h) : m1(d[a], h);
      kk += term;
    }
    tK[idx] = kk;
    tM[idx] = mm;
    tA[idx] = kk + weight_entry(g, *vs, t, tn);
  }
}

// The table of the mass matrix weighted by W (M_W, the derivative of A with
// respect to a parameter of V when W = dV/dtheta).
__global__ void k_build_wtable(Geo g, const VSpec* __restrict__ ws, double* __restrict__ tW) {
  const long total = g.tsize * g.ntaps;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x)
    tW[idx] = weight_entry(g, *ws, (int)(idx / g.tsize), idx % g.tsize);
}

void launch_build_wtable(const ddeig_problem* P, const VSpec* dws, double* tW, hipStream_t s) {
  const long total = P->g.tsize * P->g.ntaps;
  const int blocks = (int)std::min<long>((total + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_build_wtable, dim3(blocks), dim3(kBlock), 0, s, P->g, dws, tW);
}

__global__ void k_shift_table(long total, const double* __restrict__ tA,
                              const double* __restrict__ tM, double sigma,
                              double* __restrict__ tAs) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x)
    tAs[i] = tA[i] - sigma * tM[i];
}

void launch_build_tables(const ddeig_problem* P, hipStream_t s) {
  const long total = P->g.tsize * P->g.ntaps;
  const int blocks = (int)std::min<long>((total + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_build_tables, dim3(blocks), dim3(kBlock), 0, s, P->g, P->dVS, P->tabK,
                     P->tabM, P->tabA);
}

void launch_shift_table(const ddeig_problem* P, hipStream_t s) {
  const long total = P->g.tsize * P->g.ntaps;
  const int blocks = (int)std::min<long>((total + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_shift_table, dim3(blocks), dim3(kBlock), 0, s, total, P->tabA, P->tabM,
                     P->sigma, P->tabAs);
}

// y = T x over all interior unknowns of Omega_L, as an LDS-staged tile sweep.
// A workgroup takes a TX x TY (x TZ) box of unknowns at a time: it stages the
// box plus a one-node halo of the input in LDS (coalesced row loads; nodes on
// the Dirichlet boundary or outside Omega_L are staged as zero, which removes
// their taps), then each wave applies the 3^D stencil to whole rows of the box
// from LDS.  Lane l owns the x1 positions l + 64 s of a row; when n_e divides
// 64 these share one cell-local position, so the row's 3^D table coefficients
// are loaded once per lane and reused across the 64-node strides.  Taps are
// added in the order t = 0 .. 3^D - 1 for every node.
//
// MODE 1 fuses the direction update of preconditioned CG (§3,
// eq:cg-energy-norm-error-reduction): the staged vector is
// p_k = z_{k-1} + beta_k p_{k-1}, beta_k = rho_{k-1} / rho_{k-2} (p_1 = z_0),
// with rho_{k-1} = r_{k-1}.z_{k-1} from the partial sums of the extension;
// the owned nodes of p_k are written to a second buffer (other tiles still
// read p_{k-1} in their halos), and the sweep returns q = A_sigma p_k with the
// partials of p_k.q.  A non-positive rho ends CG with a breakdown.
template <int D>
struct TileShape;
template <>
struct TileShape<2> {
  static constexpr int TX = 256, TY = 8, TZ = 1;
};
template <>
struct TileShape<3> {
  static constexpr int TX = 256, TY = 1, TZ = 4;
};

template <int D, int MODE>
__global__ void __launch_bounds__(kBlock) k_stencil(Geo g, const double* __restrict__ T,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ pold,
                                                    double* __restrict__ pnew,
                                                    double* __restrict__ y, DirArgs dir,
                                                    int use_dot, Red dot, int use_sum, Red sum) {
  constexpr int TX = TileShape<D>::TX, TY = TileShape<D>::TY, TZ = TileShape<D>::TZ;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = D == 3 ? TZ + 2 : 1;
  constexpr int NT = D == 2 ? 9 : 27;
  constexpr int RX = TX / 64;
  __shared__ double sv[HX * HY * HZ];
  double beta = 0.0;
  if constexpr (MODE == 1) {
    const double rho = sum_partials(dir.rz.part, dir.rz.np);
    if (dir.st->done) return;
    if (!(rho > 0.0) || !(rho > dir.st->rz_floor)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        dir.st->done = 3;
        dir.st->iters = dir.k - 1;
      }
      return;
    }
    if (dir.k > 1) beta = rho / dir.st->rho[(dir.k - 2) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) dir.st->rho[(dir.k - 1) & 1] = rho;
  }
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2];
  const long N01 = (long)N0 * N1;
  const int nbx = (N0 + TX - 1) / TX, nby = (N1 + TY - 1) / TY;
  const int nbz = D == 3 ? (N2 + TZ - 1) / TZ : 1;
  const long ntiles = (long)nbx * nby * nbz;
  const long tsize = g.tsize;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc = 0.0, accs = 0.0;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int bx = (int)(tile % nbx);
    const long rest = tile / nbx;
    const int by = (int)(rest % nby), bz = (int)(rest / nby);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    __syncthreads();  // the previous tile's reads of sv are complete
    for (int e = threadIdx.x; e < HX * HY * HZ; e += kBlock) {
      const int ex = e % HX, er = e / HX;
      const int ey = er % HY, ez = er / HY;
      const int gx = x0 - 1 + ex, gy = y0 - 1 + ey, gz = D == 3 ? z0 - 1 + ez : 0;
      double v = 0.0;
      if (gx >= 0 && gx < N0 && gy >= 0 && gy < N1 && gz >= 0 && gz < N2) {
        const long k = gx + (long)N0 * gy + N01 * gz;
        v = x[k];
        if constexpr (MODE == 1) {
          if (dir.k > 1) v += beta * pold[k];
          const bool own = ex >= 1 && ex <= TX && ey >= 1 && ey <= TY &&
                           (D == 2 || (ez >= 1 && ez <= TZ));
          if (own) pnew[k] = v;
        }
      }
      sv[e] = v;
    }
    __syncthreads();
    // rows w, w + 4, ... of the tile (a static loop, so cpre stays in registers)
#pragma unroll
    for (int jr = 0; jr < TY * TZ / (kBlock / 64); ++jr) {
      const int row = w + (kBlock / 64) * jr;
      const int ty = row % TY, tz = row / TY;
      const int gy = y0 + ty, gz = z0 + tz;
      if (gy >= N1 || (D == 3 && gz >= N2)) continue;
      const int j1 = g.isx[1] ? (int)((unsigned)(gy + 1) - g.ne * fdiv((unsigned)(gy + 1), g.fne)) : gy;
      int j2 = 0;
      if constexpr (D == 3)
        j2 = g.isx[2] ? (int)((unsigned)(gz + 1) - g.ne * fdiv((unsigned)(gz + 1), g.fne)) : gz;
      const long trow = (long)g.P[0] * (j1 + (long)g.P[1] * j2);
      double c[NT];
      long tn_prev = -1;
#pragma unroll
      for (int s = 0; s < RX; ++s) {
        const int gx = x0 + lane + 64 * s;
        if (gx >= N0) continue;
        const int j0 = (int)((unsigned)(gx + 1) - g.ne * fdiv((unsigned)(gx + 1), g.fne));
        const long tn = j0 + trow;
        if (tn != tn_prev) {
#pragma unroll
          for (int t = 0; t < NT; ++t) c[t] = T[t * tsize + tn];
          tn_prev = tn;
        }
        const int cx = lane + 64 * s + 1;
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int d0 = t % 3 - 1, d1 = (t / 3) % 3 - 1, d2 = D == 2 ? 0 : t / 9 - 1;
          a += c[t] * sv[(cx + d0) + HX * ((ty + 1 + d1) + HY * (D == 3 ? tz + 1 + d2 : 0))];
        }
        const long k = gx + (long)N0 * gy + N01 * gz;
        y[k] = a;
        acc += sv[cx + HX * ((ty + 1) + HY * (D == 3 ? tz + 1 : 0))] * a;
        accs += a;
      }
    }
  }
  if (use_dot) write_partial(acc, dot.part);
  if (use_sum) write_partial(accs, sum.part);
}

// Workgroup b runs on XCD b mod 8 (round-robin dispatch): XCD k takes the
// k-th contiguous eighth of the n tiles, so that neighbouring tiles, which
// read each other's nodes as halo, share one L2.
__device__ __forceinline__ int xcd_slab(int b, int n) {
  const int per = n / 8, rem = n % 8, k = b % 8, i = b / 8;
  return (k < rem ? k * (per + 1) : rem * (per + 1) + (k - rem) * per) + i;
}

// The 3-D sweep with one 256 x 1 x 4 tile per workgroup: wave w takes the row
// z = z0 + w, lane l its nodes x0 + l + 64 s (s < 4).  When n_e divides 64 the
// four nodes of a lane share one cell-local position, so the 27 table
// coefficients are loaded once for four nodes: the table, not the vector, is
// what the 3-D sweep reads most.  Tiles are numbered with z fastest, then the
// one of x, y with fewer tiles, then the other, and handed out by xcd_slab, so
// an XCD holds a slab of whole planes of tiles across the two short tile
// directions and most halo reads hit its L2.  The halo staging is
// unrolled in rounds of 8 entries per thread, all loads of a round in flight
// together.  Arithmetic and tap order per node are those of k_stencil<3, MODE>;
// the block partials are stored by workgroup.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_stencil3d(Geo g, const double* __restrict__ T,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ pold,
                                                      double* __restrict__ pnew,
                                                      double* __restrict__ y, DirArgs dir,
                                                      int use_dot, Red dot, int use_sum, Red sum) {
  constexpr int TX = TileShape<3>::TX, TY = TileShape<3>::TY, TZ = TileShape<3>::TZ;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, NH = HX * HY * HZ;
  constexpr int RX = TX / 64, NR = TY * TZ / (kBlock / 64);  // strides per lane, rows per wave
  constexpr int NS = (NH + kBlock - 1) / kBlock, SB = 8;    // staged entries per thread, per round
  static_assert(TX % 64 == 0 && (TY * TZ) % (kBlock / 64) == 0, "rows of whole waves");
  __shared__ double sv[NH];
  double beta = 0.0;
  if constexpr (MODE == 1) {
    const double rho = sum_partials(dir.rz.part, dir.rz.np);
    if (dir.st->done) return;
    if (!(rho > 0.0) || !(rho > dir.st->rz_floor)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        dir.st->done = 3;
        dir.st->iters = dir.k - 1;
      }
      return;
    }
    if (dir.k > 1) beta = rho / dir.st->rho[(dir.k - 2) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) dir.st->rho[(dir.k - 1) & 1] = rho;
  }
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2];
  const long N01 = (long)N0 * N1;
  const int nbx = (N0 + TX - 1) / TX, nby = (N1 + TY - 1) / TY, nbz = (N2 + TZ - 1) / TZ;
  const int tile = xcd_slab(blockIdx.x, nbx * nby * nbz);
  const int bz = tile % nbz, rest = tile / nbz;
  const bool xmid = nbx <= nby;  // the shorter of x, y runs second fastest
  const int bx = xmid ? rest % nbx : rest / nby, by = xmid ? rest / nbx : rest % nby;
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
  const long tsize = g.tsize;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int s0 = 0; s0 < NS; s0 += SB) {
    double v[SB], vo[SB];
    long kk[SB];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = threadIdx.x + kBlock * (s0 + u);
      const int ex = e % HX, er = e / HX, ey = er % HY, ez = er / HY;
      const int gx = x0 - 1 + ex, gy = y0 - 1 + ey, gz = z0 - 1 + ez;
      const bool in = e < NH && gx >= 0 && gx < N0 && gy >= 0 && gy < N1 && gz >= 0 && gz < N2;
      kk[u] = in ? gx + (long)N0 * gy + N01 * gz : -1;
      v[u] = in ? x[kk[u]] : 0.0;
      if constexpr (MODE == 1) vo[u] = (in && dir.k > 1) ? pold[kk[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = threadIdx.x + kBlock * (s0 + u);
      if (e >= NH) continue;
      double val = v[u];
      if constexpr (MODE == 1) {
        if (kk[u] >= 0) {
          if (dir.k > 1) val += beta * vo[u];
          const int ex = e % HX, er = e / HX, ey = er % HY, ez = er / HY;
          if (ex >= 1 && ex <= TX && ey >= 1 && ey <= TY && ez >= 1 && ez <= TZ)
            pnew[kk[u]] = val;
        }
      }
      sv[e] = val;
    }
  }
  __syncthreads();
  double acc = 0.0, accs = 0.0;
#pragma unroll
  for (int jr = 0; jr < NR; ++jr) {
    const int row = w + (kBlock / 64) * jr;
    const int ty = row % TY, tz = row / TY;
    const int gy = y0 + ty, gz = z0 + tz;
    if (gy >= N1 || gz >= N2) continue;
    const int j1 = g.isx[1] ? (int)((unsigned)(gy + 1) - g.ne * fdiv((unsigned)(gy + 1), g.fne)) : gy;
    const int j2 = g.isx[2] ? (int)((unsigned)(gz + 1) - g.ne * fdiv((unsigned)(gz + 1), g.fne)) : gz;
    const long trow = (long)g.P[0] * (j1 + (long)g.P[1] * j2);
    double c[27];
    long tn_prev = -1;
#pragma unroll
    for (int s = 0; s < RX; ++s) {
      const int gx = x0 + lane + 64 * s;
      if (gx >= N0) continue;
      const int j0 = (int)((unsigned)(gx + 1) - g.ne * fdiv((unsigned)(gx + 1), g.fne));
      const long tn = j0 + trow;
      if (tn != tn_prev) {
#pragma unroll
        for (int t = 0; t < 27; ++t) c[t] = T[t * tsize + tn];
        tn_prev = tn;
      }
      const int cx = lane + 64 * s + 1;
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int d0 = t % 3 - 1, d1 = (t / 3) % 3 - 1, d2 = t / 9 - 1;
        a += c[t] * sv[(cx + d0) + HX * ((ty + 1 + d1) + HY * (tz + 1 + d2))];
      }
      if constexpr (MODE == 0) __builtin_nontemporal_store(a, &y[gx + (long)N0 * gy + N01 * gz]);
      else y[gx + (long)N0 * gy + N01 * gz] = a;
      acc += sv[cx + HX * ((ty + 1) + HY * (tz + 1))] * a;
      accs += a;
    }
  }
  if (use_dot) write_partial(acc, dot.part);
  if (use_sum) write_partial(accs, sum.part);
}

// The 2-D sweep when n_e divides 64 (every lane keeps one cell-local x
// position across its 64-node strides): one 256 x 8 tile per workgroup, the
// 2 x 9 table coefficients of the thread's rows loaded before the staging so
// that both latency rounds overlap, and 32-bit tile-local index arithmetic
// (fewer registers, more resident waves).  Same arithmetic and tap order as
// k_stencil<2, MODE>.
// The body takes the block's tile index `bid` (blockIdx.x of a single
// problem, or the block's index within its instance in a grouped launch).
// YFAST numbers the tiles y fastest: with bid = xcd_slab(blockIdx.x) an XCD
// then holds a run of whole tile columns, so the halo rows a tile shares with
// its y neighbours come from that XCD's L2 instead of HBM (the grids of these
// problems are a few tiles tall and very wide).
template <int MODE, int TY = 8, bool YFAST = false>
__device__ __forceinline__ void stencil2d_body(const Geo& g, const double* __restrict__ T,
                                               const double* __restrict__ x,
                                               const double* __restrict__ pold,
                                               double* __restrict__ pnew, double* __restrict__ y,
                                               const DirArgs& dir, int use_dot, const Red& dot,
                                               int use_sum, const Red& sum, int bid) {
  constexpr int TX = 256, HX = TX + 2, HY = TY + 2, RX = TX / 64, RY = TY / 4;
  __shared__ double sv[HX * HY];
  double beta = 0.0;
  if constexpr (MODE == 1) {
    const double rho = sum_partials(dir.rz.part, dir.rz.np);
    if (dir.st->done) return;
    if (!(rho > 0.0) || !(rho > dir.st->rz_floor)) {
      if (bid == 0 && threadIdx.x == 0) {
        dir.st->done = 3;
        dir.st->iters = dir.k - 1;
      }
      return;
    }
    if (dir.k > 1) beta = rho / dir.st->rho[(dir.k - 2) & 1];
    if (bid == 0 && threadIdx.x == 0) dir.st->rho[(dir.k - 1) & 1] = rho;
  }
  const int N0 = g.N[0], N1 = g.N[1];
  const int nbx = (N0 + TX - 1) / TX, nby = (N1 + TY - 1) / TY;
  const int bx = YFAST ? bid / nby : bid % nbx, by = YFAST ? bid % nby : bid / nbx;
  const int x0 = bx * TX, y0 = by * TY;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // cell-local x position of the lane (the same for all its strides)
  const int j0 = (int)((unsigned)(x0 + lane + 1) - g.ne * fdiv((unsigned)(x0 + lane + 1), g.fne));
  const long tsize = g.tsize;
  double c[RY][9];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const int gy = min(y0 + w + 4 * j, N1 - 1);
    const double* tp = T + j0 + g.P[0] * gy;
#pragma unroll
    for (int t = 0; t < 9; ++t) c[j][t] = tp[t * tsize];
  }
  // the halo staging, unrolled in rounds of SB entries per thread so that all
  // loads of a round are in flight together
  constexpr int NH = HX * HY, NS = (NH + kBlock - 1) / kBlock, SB = 8;
  const long base = (long)N0 * y0 + x0;
#pragma unroll
  for (int s0 = 0; s0 < NS; s0 += SB) {
    double v[SB], vo[SB];
    long off[SB];
    bool in[SB];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = threadIdx.x + kBlock * (s0 + u);
      const int ex = e % HX, ey = e / HX;
      const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
      in[u] = e < NH && gx >= 0 && gx < N0 && gy >= 0 && gy < N1;
      off[u] = (long)N0 * (ey - 1) + (ex - 1);
      v[u] = in[u] ? x[base + off[u]] : 0.0;
      if constexpr (MODE == 1) vo[u] = (in[u] && dir.k > 1) ? pold[base + off[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = threadIdx.x + kBlock * (s0 + u);
      if (e >= NH) continue;
      double val = v[u];
      if constexpr (MODE == 1) {
        if (in[u]) {
          if (dir.k > 1) val += beta * vo[u];
          const int ex = e % HX, ey = e / HX;
          if (ex >= 1 && ex <= TX && ey >= 1 && ey <= TY) pnew[base + off[u]] = val;
        }
      }
      sv[e] = val;
    }
  }
  __syncthreads();
  double acc = 0.0, accs = 0.0;
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const int ty = w + 4 * j, gy = y0 + ty;
    if (gy >= N1) continue;
#pragma unroll
    for (int s = 0; s < RX; ++s) {
      const int gx = x0 + lane + 64 * s;
      if (gx >= N0) continue;
      const int cx = lane + 64 * s + 1;
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) a += c[j][t] * sv[(cx + t % 3 - 1) + HX * (ty + t / 3)];
      // the plain sweep's result is not read again by the sweep: streamed past
      // the caches (non-temporal), which helps when the vectors exceed them
      if constexpr (MODE == 0) __builtin_nontemporal_store(a, &y[gx + (long)N0 * gy]);
      else y[gx + (long)N0 * gy] = a;
      acc += sv[cx + HX * (ty + 1)] * a;
      accs += a;
    }
  }
  if (use_dot) write_partial_at(acc, dot.part, bid);
  if (use_sum) write_partial_at(accs, sum.part, bid);
}

template <int MODE, int TY>
__global__ void __launch_bounds__(kBlock) k_stencil2d(Geo g, const double* __restrict__ T,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ pold,
                                                      double* __restrict__ pnew,
                                                      double* __restrict__ y, DirArgs dir,
                                                      int use_dot, Red dot, int use_sum, Red sum) {
  stencil2d_body<MODE, TY, true>(g, T, x, pold, pnew, y, dir, use_dot, dot, use_sum, sum,
                                 xcd_slab(blockIdx.x, gridDim.x));
}

// The 2-D sweep of wide grids (n_e dividing 64): one wave per workgroup owns
// kMarchX = 512 columns, lane l the columns x0 + l + 64 s (s < 8), which share
// one cell-local position and so every table coefficient the lane loads, and
// marches through all N1 rows.  With input row k staged in LDS (plus its two
// halo columns) the lane adds taps 6..8 to output row k - 1, taps 3..5 to row
// k and taps 0..2 to row k + 1; every output so receives its taps in the
// order t = 0..8 of the tile sweep, from the same values, and equals the tile
// sweep's result bit for bit.  Row k - 1 is then complete and stored.  Each
// input row is read once (tiles re-read their halo rows), and the next row
// and the next step's coefficients are loaded one step ahead into registers:
// this is the sweep that streams wide grids at near-copy bandwidth.
// Loads use clamped in-range addresses; the masks (Dirichlet ends, columns
// past N0) are applied when a row is staged.  MODE 1 stages
// p_k = z + beta p_{k-1} as the tile sweep does, writes the owned entries of
// p_k and forms the partials of p_k.q; one partial per workgroup.
constexpr int kMarchRX = 8, kMarchX = 64 * kMarchRX;

template <int MODE>
__global__ void __launch_bounds__(64) k_stencil2d_march(Geo g, const double* __restrict__ T,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ pold,
                                                        double* __restrict__ pnew,
                                                        double* __restrict__ y, DirArgs dir,
                                                        int use_dot, Red dot, int use_sum, Red sum) {
  constexpr int RX = kMarchRX, TX = kMarchX, HX = TX + 2;
  __shared__ double rows[2][HX];
  double beta = 0.0;
  if constexpr (MODE == 1) {
    const double rho = sum_partials<64>(dir.rz.part, dir.rz.np);
    if (dir.st->done) return;
    if (!(rho > 0.0) || !(rho > dir.st->rz_floor)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        dir.st->done = 3;
        dir.st->iters = dir.k - 1;
      }
      return;
    }
    if (dir.k > 1) beta = rho / dir.st->rho[(dir.k - 2) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) dir.st->rho[(dir.k - 1) & 1] = rho;
  }
  const bool upd = MODE == 1 && dir.k > 1;
  const int N0 = g.N[0], N1 = g.N[1];
  const int x0 = xcd_slab(blockIdx.x, gridDim.x) * TX;
  const int lane = threadIdx.x;
  const int j0 = (int)((unsigned)(x0 + lane + 1) - g.ne * fdiv((unsigned)(x0 + lane + 1), g.fne));
  const long tsize = g.tsize;
  const int P0 = g.P[0];
  // lane 0 stages the halo column x0 - 1, lane 1 the column x0 + TX
  const int hx = lane == 0 ? x0 - 1 : x0 + TX;
  const bool hin = lane < 2 && hx >= 0 && hx < N0;
  const long hxc = hin ? hx : x0;
  bool in[RX];
  long xs[RX];
#pragma unroll
  for (int s = 0; s < RX; ++s) {
    in[s] = x0 + lane + 64 * s < N0;
    xs[s] = in[s] ? x0 + lane + 64 * s : x0;
  }
  double bx[RX + 1], bp[RX + 1];
  auto load_row = [&](int r) {
    const long ro = (long)N0 * min(r, N1 - 1);
#pragma unroll
    for (int s = 0; s < RX; ++s) bx[s] = x[xs[s] + ro];
    bx[RX] = x[hxc + ro];
    if (upd) {
#pragma unroll
      for (int s = 0; s < RX; ++s) bp[s] = pold[xs[s] + ro];
      bp[RX] = pold[hxc + ro];
    }
  };
  // coefficients of the taps that input row k gives to output rows k - 1, k,
  // k + 1 (row indices clamped: the sums of rows -1 and N1 are never used)
  auto coef = [&](int k, double* c) {
    const double* tm = T + j0 + (long)P0 * max(k - 1, 0);
    const double* t0 = T + j0 + (long)P0 * min(k, N1 - 1);
    const double* tp = T + j0 + (long)P0 * min(k + 1, N1 - 1);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      c[t] = tm[(6 + t) * tsize];
      c[3 + t] = t0[(3 + t) * tsize];
      c[6 + t] = tp[t * tsize];
    }
  };
  double cn[9];
  load_row(0);
  coef(0, cn);
  double am[RX], a0[RX], ap[RX], vp[RX];
#pragma unroll
  for (int s = 0; s < RX; ++s) {
    am[s] = 0.0;
    a0[s] = 0.0;
    ap[s] = 0.0;
    vp[s] = 0.0;
  }
  double acc = 0.0, accs = 0.0;
  for (int k = 0; k < N1; ++k) {
    double* rw = rows[k & 1];
    double vc[RX];
#pragma unroll
    for (int s = 0; s < RX; ++s) {
      double v = bx[s];
      if (upd) v += beta * bp[s];
      v = in[s] ? v : 0.0;
      vc[s] = v;
      rw[1 + lane + 64 * s] = v;
      if constexpr (MODE == 1) {
        if (in[s]) pnew[xs[s] + (long)N0 * k] = v;
      }
    }
    if (lane < 2) {
      double v = bx[RX];
      if (upd) v += beta * bp[RX];
      rw[lane == 0 ? 0 : HX - 1] = hin ? v : 0.0;
    }
    double c[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) c[t] = cn[t];
    coef(k + 1, cn);
    load_row(k + 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RX; ++s) {
      const int cx = 1 + lane + 64 * s;
      const double vl = rw[cx - 1], vm = rw[cx], vr = rw[cx + 1];
      if (k > 0) {
        am[s] += c[0] * vl;
        am[s] += c[1] * vm;
        am[s] += c[2] * vr;
      }
      a0[s] += c[3] * vl;
      a0[s] += c[4] * vm;
      a0[s] += c[5] * vr;
      if (k + 1 < N1) {
        ap[s] += c[6] * vl;
        ap[s] += c[7] * vm;
        ap[s] += c[8] * vr;
      }
    }
    if (k > 0) {
#pragma unroll
      for (int s = 0; s < RX; ++s) {
        if (!in[s]) continue;
        double* yp = &y[xs[s] + (long)N0 * (k - 1)];
        if constexpr (MODE == 0) __builtin_nontemporal_store(am[s], yp);
        else *yp = am[s];
        acc += vp[s] * am[s];
        accs += am[s];
      }
    }
#pragma unroll
    for (int s = 0; s < RX; ++s) {
      am[s] = a0[s];
      a0[s] = ap[s];
      ap[s] = 0.0;
      vp[s] = vc[s];
    }
  }
#pragma unroll
  for (int s = 0; s < RX; ++s) {
    if (!in[s]) continue;
    double* yp = &y[xs[s] + (long)N0 * (N1 - 1)];
    if constexpr (MODE == 0) __builtin_nontemporal_store(am[s], yp);
    else *yp = am[s];
    acc += vp[s] * am[s];
    accs += am[s];
  }
  if (use_dot) write_partial<64>(acc, dot.part);
  if (use_sum) write_partial<64>(accs, sum.part);
}

// The 3-D sweep of wide grids (n_e dividing 32): a workgroup owns a 256 x 8
// block of (x, y) lines and marches through all N2 planes.  Lane l of wave w
// takes the row y0 + 2 w + l / 32 and the columns x0 + l % 32 + 32 s (s < 8),
// which share one cell-local position, so each of the 27 table coefficients a
// lane loads per plane serves eight outputs.  With input plane k staged in LDS
// (the block plus a one-node halo in x and y) every lane adds taps 18..26 to
// its outputs in plane k - 1, taps 9..17 to plane k and taps 0..8 to plane
// k + 1: each output receives its taps in the order t = 0..26 of the tile
// sweep, from the same values, and equals the tile sweep's result bit for
// bit.  Plane k - 1 is then complete and stored.  Each plane of the block is
// read once and the next plane is loaded one step ahead; the loads are buffer
// loads whose per-lane offsets stay in one register each (the tap and plane
// offsets ride in scalar registers), from clamped in-range offsets, the masks
// applied when a plane is staged.  MODE 1 stages p_k = z + beta p_{k-1} as
// the tile sweep does, writes the owned entries of p_k and forms the partials
// of p_k.q.  One partial per workgroup; needs 8 N < 2^31 (stencil3d_march).
constexpr int kPlaneTX = 256, kPlaneTY = 8;

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_stencil3d_march(Geo g, const double* __restrict__ T,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ pold,
                                                            double* __restrict__ pnew,
                                                            double* __restrict__ y, DirArgs dir,
                                                            int use_dot, Red dot, int use_sum, Red sum) {
  constexpr int TX = kPlaneTX, TY = kPlaneTY, HX = TX + 2, HY = TY + 2, NH = HX * HY, RX = 8;
  constexpr int NS = (NH + kBlock - 1) / kBlock;
  static_assert(TY == 2 * (kBlock / 64) && TX == 32 * RX, "two rows per wave, 32 lanes per row");
  __shared__ double pl[2][NH];
  double beta = 0.0;
  if constexpr (MODE == 1) {
    const double rho = sum_partials(dir.rz.part, dir.rz.np);
    if (dir.st->done) return;
    if (!(rho > 0.0) || !(rho > dir.st->rz_floor)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        dir.st->done = 3;
        dir.st->iters = dir.k - 1;
      }
      return;
    }
    if (dir.k > 1) beta = rho / dir.st->rho[(dir.k - 2) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) dir.st->rho[(dir.k - 1) & 1] = rho;
  }
  const bool upd = MODE == 1 && dir.k > 1;
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2];
  const long N01 = (long)N0 * N1;
  const int nby = (N1 + TY - 1) / TY;
  const int bid = xcd_slab(blockIdx.x, gridDim.x);
  const int x0 = (bid / nby) * TX, y0 = (bid % nby) * TY;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int xl = lane & 31, ty = 2 * w + (lane >> 5);
  const unsigned tsz8 = (unsigned)(g.tsize * 8);
  const unsigned pp8 = (unsigned)(g.P[0] * g.P[1] * 8);
  const unsigned pl8 = (unsigned)(N01 * 8);
  const int nbytes = (int)(N01 * N2 * 8);
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void*)pold, (short)0, nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc((void*)T, (short)0,
                                                                      (int)(27 * g.tsize * 8), 0x00020000);
  const int j0 = (int)((unsigned)(x0 + xl + 1) - g.ne * fdiv((unsigned)(x0 + xl + 1), g.fne));
  const int gy = y0 + ty;
  const bool rowin = gy < N1;
  const int gyc = min(gy, N1 - 1);
  const int j1 = g.isx[1] ? (int)((unsigned)(gyc + 1) - g.ne * fdiv((unsigned)(gyc + 1), g.fne)) : gyc;
  const unsigned coff = (unsigned)(j0 + g.P[0] * j1) * 8u;
  // staging slots of this thread: in-plane offsets (0 when outside the grid),
  // in-grid and owned masks
  unsigned voff[NS];
  unsigned inm = 0, own = 0;
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int e = threadIdx.x + kBlock * u;
    const int ex = e % HX, ey = e / HX;
    const int gx = x0 - 1 + ex, gyy = y0 - 1 + ey;
    const bool in = e < NH && gx >= 0 && gx < N0 && gyy >= 0 && gyy < N1;
    voff[u] = in ? (unsigned)(gx + N0 * gyy) * 8u : 0u;
    inm |= in ? (1u << u) : 0u;
    own |= (in && ex >= 1 && ex <= TX && ey >= 1 && ey <= TY) ? (1u << u) : 0u;
  }
  double nx[NS], np[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    nx[u] = buf_load(rx, voff[u], 0);
    if (upd) np[u] = buf_load(rp, voff[u], 0);
  }
  double am[RX], a0[RX], ap[RX], vc[RX], vp[RX];
#pragma unroll
  for (int s = 0; s < RX; ++s) {
    am[s] = 0.0;
    a0[s] = 0.0;
    ap[s] = 0.0;
    vp[s] = 0.0;
  }
  double acc = 0.0, accs = 0.0;
  for (int k = 0; k < N2; ++k) {
    double* P = pl[k & 1];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = threadIdx.x + kBlock * u;
      if (e >= NH) continue;
      double v = nx[u];
      if (upd) v += beta * np[u];
      v = (inm >> u) & 1 ? v : 0.0;
      P[e] = v;
      if constexpr (MODE == 1) {
        if ((own >> u) & 1) pnew[voff[u] / 8 + N01 * k] = v;
      }
    }
    if (k + 1 < N2) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        nx[u] = buf_load(rx, voff[u], pl8 * (k + 1));
        if (upd) np[u] = buf_load(rp, voff[u], pl8 * (k + 1));
      }
    }
    // coefficients of the taps plane k gives to planes k - 1, k, k + 1 (plane
    // indices clamped: the sums of planes -1 and N2 are never used)
    double c[27];
    {
      const unsigned om = pp8 * (unsigned)max(k - 1, 0), o0 = pp8 * (unsigned)k,
                     op = pp8 * (unsigned)min(k + 1, N2 - 1);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        c[t] = buf_load(rt, coff, (18 + t) * tsz8 + om);
        c[9 + t] = buf_load(rt, coff, (9 + t) * tsz8 + o0);
        c[18 + t] = buf_load(rt, coff, t * tsz8 + op);
      }
    }
    __syncthreads();
    // MODE 0 takes the columns in two halves with a barrier between them
    // (outside the divergent row test): left to itself the compiler issues
    // all 72 LDS reads of a plane before the first FMA and the kernel needs
    // ~270 VGPRs (one wave per SIMD); by halves it needs ~200 and two waves
    // fit (62,979,135 unknowns: 411 -> 350 us).  MODE 1 holds the previous
    // direction's plane as well and stays near 270 VGPRs either way; the
    // barrier only costs it time, so it keeps one group.
    constexpr int NG = MODE == 0 ? 2 : 1;
#pragma unroll
    for (int h = 0; h < NG; ++h) {
      if (h > 0) __syncthreads();
      if (rowin) {
#pragma unroll
        for (int s = h * (RX / NG); s < (h + 1) * (RX / NG); ++s) {
          const int cx = xl + 32 * s + 1;
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            const double v = P[(cx + t % 3 - 1) + HX * (ty + t / 3)];
            if (t == 4) vc[s] = v;
            am[s] += c[t] * v;
            a0[s] += c[9 + t] * v;
            ap[s] += c[18 + t] * v;
          }
        }
      }
    }
    if (rowin) {
      if (k > 0) {
#pragma unroll
        for (int s = 0; s < RX; ++s) {
          const int gx = x0 + xl + 32 * s;
          if (gx >= N0) continue;
          double* yp = &y[gx + (long)N0 * gy + N01 * (k - 1)];
          if constexpr (MODE == 0) __builtin_nontemporal_store(am[s], yp);
          else *yp = am[s];
          acc += vp[s] * am[s];
          accs += am[s];
        }
      }
#pragma unroll
      for (int s = 0; s < RX; ++s) {
        am[s] = a0[s];
        a0[s] = ap[s];
        ap[s] = 0.0;
        vp[s] = vc[s];
      }
    }
  }
  if (rowin) {
#pragma unroll
    for (int s = 0; s < RX; ++s) {
      const int gx = x0 + xl + 32 * s;
      if (gx >= N0) continue;
      double* yp = &y[gx + (long)N0 * gy + N01 * (N2 - 1)];
      if constexpr (MODE == 0) __builtin_nontemporal_store(am[s], yp);
      else *yp = am[s];
      acc += vp[s] * am[s];
      accs += am[s];
    }
  }
  if (use_dot) write_partial(acc, dot.part);
  if (use_sum) write_partial(accs, sum.part);
}

// Grouped direction update + A_sigma p of PCG iteration k over the instances
// of a batch: block b runs tile map[b].y of instance map[b].x.
__global__ void __launch_bounds__(kBlock) k_b_stencil_dir(const InstDev* __restrict__ I,
                                                          const int2* __restrict__ map, int k) {
  const int2 m = map[blockIdx.x];
  const InstDev& d = I[m.x];
  const DirArgs dir{d.st, k, d.rz};
  const Red none{nullptr, 0, nullptr};
  // the instance's tile rows, as in its own sweep (uniform per block)
  if (d.sty == 4)
    stencil2d_body<1, 4>(d.g, d.tabAs, d.z, d.pp[(k - 1) & 1], d.pp[k & 1], d.q, dir, 1, d.gam, 0,
                         none, m.y);
  else
    stencil2d_body<1, 8>(d.g, d.tabAs, d.z, d.pp[(k - 1) & 1], d.pp[k & 1], d.q, dir, 1, d.gam, 0,
                         none, m.y);
}

void launch_b_stencil_dir(const InstDev* I, const BlockMap& bm, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_b_stencil_dir, dim3(bm.nblocks), dim3(kBlock), 0, s, I, bm.map, k);
}

// Grouped plain sweeps of the batch's outer inverse iteration over the
// instances with act[j] != 0 (block b runs tile map[b].y of instance
// map[b].x): which 0: w = M x; 1: Mu = M u (into z) with the partials of u.Mu
// and sum(Mu); 2: q = A_sigma x with the partials of x.q.
__global__ void __launch_bounds__(kBlock) k_b_stencil_plain(const InstDev* __restrict__ I,
                                                            const int2* __restrict__ map,
                                                            const int* __restrict__ act, int which) {
  const int2 m = map[blockIdx.x];
  if (!act[m.x]) return;
  const InstDev& d = I[m.x];
  const Red none{nullptr, 0, nullptr};
  const DirArgs nodir{nullptr, 0, none};
  const double* T = which == 2 ? d.tabAs : d.tabM;
  const double* xin = which == 1 ? d.x : d.xo;
  double* yout = which == 0 ? d.w : (which == 1 ? d.z : d.q);
  const Red dot = which == 1 ? d.nm_uMu : d.nm_xq;
  const int use_dot = which != 0, use_sum = which == 1;
  if (d.sty == 4)
    stencil2d_body<0, 4>(d.g, T, xin, nullptr, nullptr, yout, nodir, use_dot, dot, use_sum,
                         d.nm_sum, m.y);
  else
    stencil2d_body<0, 8>(d.g, T, xin, nullptr, nullptr, yout, nodir, use_dot, dot, use_sum,
                         d.nm_sum, m.y);
}

void launch_b_stencil_plain(const InstDev* I, const BlockMap& bm, const int* act, int which,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_b_stencil_plain, dim3(bm.nblocks), dim3(kBlock), 0, s, I, bm.map, act,
                     which);
}

// Rows of the 2-D sweep's tiles (n_e dividing 64): 4 while 4-row tiles number
// at most 1024 (one partial each), else 8.  Small grids, whose vectors sit in
// the Infinity Cache and whose sweep is latency-bound, get twice the
// workgroups (config 2: 1024 tiles, 7.2 -> 5.9 us per sweep).
int stencil2d_ty(const Geo& g) {
  const long t4 = (long)((g.N[0] + 255) / 256) * ((g.N[1] + 3) / 4);
  return t4 <= kMaxRed ? 4 : 8;
}

static bool stencil2d_fast(const Geo& g) { return g.D == 2 && 64 % g.ne == 0; }

// The row march serves 2-D grids with n_e dividing 64 whose width gives at
// least 1024 of its 512-column workgroups (ddeig_options.sweep 0), or on
// request (sweep 2); sweep 1 keeps the tiles (in 3-D as well).
static bool stencil2d_march(const ddeig_problem* P) {
  const Geo& g = P->g;
  if (!stencil2d_fast(g) || P->opt.sweep == 1) return false;
  return P->opt.sweep == 2 || (g.N[0] + kMarchX - 1) / kMarchX >= 1024;
}

// The plane march serves 3-D grids with n_e dividing 32 whose (x, y) extent
// gives at least 1024 of its 256 x 8 blocks (sweep 0), or on request (sweep 2);
// its buffer offsets need 8 N < 2^31.
static long stencil3d_march_blocks(const Geo& g) {
  return (long)((g.N[0] + kPlaneTX - 1) / kPlaneTX) * ((g.N[1] + kPlaneTY - 1) / kPlaneTY);
}

static bool stencil3d_march(const ddeig_problem* P) {
  const Geo& g = P->g;
  if (g.D != 3 || 32 % g.ne != 0 || P->opt.sweep == 1) return false;
  if (g.n * 8 >= (1L << 31) || 27 * g.tsize * 8 >= (1L << 31)) return false;
  return P->opt.sweep == 2 || stencil3d_march_blocks(g) >= 1024;
}

// Workgroups (and block partials) of the sweep launch_stencil runs.
long stencil_blocks(const ddeig_problem* P) {
  if (stencil2d_march(P)) return (P->g.N[0] + kMarchX - 1) / kMarchX;
  if (stencil3d_march(P)) return stencil3d_march_blocks(P->g);
  return stencil_tiles(P->g);
}

long stencil_tiles(const Geo& g) {
  if (stencil2d_fast(g)) {
    const int ty = stencil2d_ty(g);
    return (long)((g.N[0] + 255) / 256) * ((g.N[1] + ty - 1) / ty);
  }
  if (g.D == 2)
    return (long)((g.N[0] + TileShape<2>::TX - 1) / TileShape<2>::TX) *
           ((g.N[1] + TileShape<2>::TY - 1) / TileShape<2>::TY);
  return (long)((g.N[0] + TileShape<3>::TX - 1) / TileShape<3>::TX) *
         ((g.N[1] + TileShape<3>::TY - 1) / TileShape<3>::TY) *
         ((g.N[2] + TileShape<3>::TZ - 1) / TileShape<3>::TZ);
}

// Sum of np block partials into out[0], in block order, by one workgroup.
__global__ void __launch_bounds__(kBig) k_reduce_partials(const double* __restrict__ part, long np,
                                                          double* __restrict__ out) {
  double v = 0.0;
  for (long i = threadIdx.x; i < np; i += kBig) v += part[i];
  v = block_sum_n<kBig>(v);
  if (threadIdx.x == 0) out[0] = v;
}

// One tile per workgroup.  Up to kMaxRed tiles the block partials go straight
// to the consumer's buffer; beyond that they go to a large per-problem buffer
// and one workgroup adds them into a single partial (np = 1).
struct TileRed {
  Red use;    // what the kernel writes
  Red final;  // what the consumers read
};

static TileRed tile_red(const ddeig_problem* P, const Red& r, long tiles, int which) {
  TileRed t{r, r};
  if (tiles <= kMaxRed) {
    t.use.np = t.final.np = (int)tiles;
  } else {
    t.use.part = P->big_part + (long)which * P->big_cap;
    t.use.np = (int)tiles;
    t.final.np = 1;
  }
  return t;
}

static void finish_tile_red(const ddeig_problem* P, const TileRed& t, hipStream_t s) {
  if (t.use.part != t.final.part)
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBig), 0, s, t.use.part,
                       (long)t.use.np, t.final.part);
}

void launch_stencil(const ddeig_problem* P, const double* tab, const double* x, double* y,
                    Red* dot, Red* sum, hipStream_t s) {
  const long tiles = stencil_blocks(P);
  const Red none{nullptr, 0, nullptr};
  const DirArgs nodir{nullptr, 0, none};
  const TileRed td = tile_red(P, dot ? *dot : none, tiles, 0);
  const TileRed ts = tile_red(P, sum ? *sum : none, tiles, 1);
  const int blocks = (int)std::max<long>(1, tiles);
  if (stencil2d_march(P)) {
    hipLaunchKernelGGL(k_stencil2d_march<0>, dim3(blocks), dim3(64), 0, s, P->g, tab, x, nullptr,
                       nullptr, y, nodir, dot ? 1 : 0, td.use, sum ? 1 : 0, ts.use);
  }
  else if (stencil3d_march(P)) {
    hipLaunchKernelGGL(k_stencil3d_march<0>, dim3(blocks), dim3(kBlock), 0, s, P->g, tab, x,
                       nullptr, nullptr, y, nodir, dot ? 1 : 0, td.use, sum ? 1 : 0, ts.use);
  }
  else if (stencil2d_fast(P->g)) {
    auto kern = stencil2d_ty(P->g) == 4 ? k_stencil2d<0, 4> : k_stencil2d<0, 8>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, P->g, tab, x, nullptr, nullptr, y,
                       nodir, dot ? 1 : 0, td.use, sum ? 1 : 0, ts.use);
  }
  else if (P->g.D == 2)
    hipLaunchKernelGGL((k_stencil<2, 0>), dim3(blocks), dim3(kBlock), 0, s, P->g, tab, x,
                       nullptr, nullptr, y, nodir, dot ? 1 : 0, td.use, sum ? 1 : 0, ts.use);
  else
    hipLaunchKernelGGL((k_stencil3d<0>), dim3(blocks), dim3(kBlock), 0, s, P->g, tab, x, nullptr,
                       nullptr, y, nodir, dot ? 1 : 0, td.use, sum ? 1 : 0, ts.use);
  if (dot) {
    finish_tile_red(P, td, s);
    *dot = td.final;
  }
  if (sum) {
    finish_tile_red(P, ts, s);
    *sum = ts.final;
  }
}

void launch_stencil_dir(const ddeig_problem* P, const double* z, const double* pold, double* pnew,
                        double* q, const DirArgs& dir, Red& gam, hipStream_t s) {
  const long tiles = stencil_blocks(P);
  const Red none{nullptr, 0, nullptr};
  const TileRed tg = tile_red(P, gam, tiles, 0);
  const int blocks = (int)std::max<long>(1, tiles);
  if (stencil2d_march(P)) {
    hipLaunchKernelGGL(k_stencil2d_march<1>, dim3(blocks), dim3(64), 0, s, P->g, P->tabAs, z,
                       pold, pnew, q, dir, 1, tg.use, 0, none);
  }
  else if (stencil3d_march(P)) {
    hipLaunchKernelGGL(k_stencil3d_march<1>, dim3(blocks), dim3(kBlock), 0, s, P->g, P->tabAs, z,
                       pold, pnew, q, dir, 1, tg.use, 0, none);
  }
  else if (stencil2d_fast(P->g)) {
    auto kern = stencil2d_ty(P->g) == 4 ? k_stencil2d<1, 4> : k_stencil2d<1, 8>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, P->g, P->tabAs, z, pold, pnew, q,
                       dir, 1, tg.use, 0, none);
  }
  else if (P->g.D == 2)
    hipLaunchKernelGGL((k_stencil<2, 1>), dim3(blocks), dim3(kBlock), 0, s, P->g, P->tabAs, z,
                       pold, pnew, q, dir, 1, tg.use, 0, none);
  else
    hipLaunchKernelGGL((k_stencil3d<1>), dim3(blocks), dim3(kBlock), 0, s, P->g, P->tabAs, z,
                       pold, pnew, q, dir, 1, tg.use, 0, none);
  finish_tile_red(P, tg, s);
  gam = tg.final;
}

// Box operator with periodic wrap in the flagged dims (the cell problem of
// eq:weak-form-cell-problem, periodic in x, Dirichlet in y).  The box vector
// uses the box's natural order (dim 0 fastest).  Partials of x.y and sum(y).
__global__ void k_box_stencil(Geo g, Box bx, const double* __restrict__ T,
                              const double* __restrict__ x, double* __restrict__ y, int use_dot,
                              Red dot, int use_sum, Red sum) {
  const long nb = (long)bx.m[0] * bx.m[1] * bx.m[2];
  double acc = 0.0, accs = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nb;
       e += (long)gridDim.x * blockDim.x) {
    int u[3] = {(int)(e % bx.m[0]), (int)((e / bx.m[0]) % bx.m[1]),
                (int)(e / ((long)bx.m[0] * bx.m[1]))};
    const long tn = table_node(g, bx.o[0] + u[0], bx.o[1] + u[1], bx.o[2] + u[2]);
    double s = 0.0;
    for (int t = 0; t < g.ntaps; ++t) {
      int d[3];
      tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
      int v[3];
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        int w = u[a] + (a < g.D ? d[a] : 0);
        if (bx.per[a]) w = (w + bx.m[a]) % bx.m[a];
        else if (w < 0 || w >= bx.m[a]) in = false;
        v[a] = w;
      }
      if (in) s += T[t * g.tsize + tn] * x[v[0] + (long)bx.m[0] * (v[1] + (long)bx.m[1] * v[2])];
    }
    y[e] = s;
    acc += x[e] * s;
    accs += s;
  }
  if (use_dot) write_partial(acc, dot.part);
  if (use_sum) write_partial(accs, sum.part);
}

void launch_box_stencil(const ddeig_problem* P, const Box& bx, const double* tab, const double* x,
                        double* y, Red* dot, Red* sum, hipStream_t s) {
  const long nb = (long)bx.m[0] * bx.m[1] * bx.m[2];
  const int blocks = red_grid(nb);
  const Red none{nullptr, 0, nullptr};
  if (dot) dot->np = blocks;
  if (sum) sum->np = blocks;
  hipLaunchKernelGGL(k_box_stencil, dim3(blocks), dim3(kBlock), 0, s, P->g, bx, tab, x, y,
                     dot ? 1 : 0, dot ? *dot : none, sum ? 1 : 0, sum ? *sum : none);
}

}  // namespace ddeig

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

// Table entries of one (table node, tap): K, M and M_V.  The loops visit the
// elements shared by the node and its neighbour in increasing element index
// and the quadrature points in a fixed order, and the shape-function product
// is formed symmetrically, so a(j, j+d) and a(j+d, j) come out bit-identical.
__global__ void k_build_tables(Geo g, const VSpec* __restrict__ vs, double* __restrict__ tK,
                               double* __restrict__ tM, double* __restrict__ tA) {
  const long total = g.tsize * g.ntaps;
  const double xi_lo = 0.5 * (1.0 - 0.57735026918962576450914878050196);
  const double xi_hi = 0.5 * (1.0 + 0.57735026918962576450914878050196);
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int t = (int)(idx / g.tsize);
    const long tn = idx % g.tsize;
    int d[3];
    tap_offsets(t, g.ntaps, d[0], d[1], d[2]);
    int j[3];
    j[0] = (int)(tn % g.P[0]);
    j[1] = (int)((tn / g.P[0]) % g.P[1]);
    j[2] = (int)(tn / ((long)g.P[0] * g.P[1]));
    const double h = g.h;
    // constant-coefficient parts
    double kk = 0.0, mm = 1.0;
    for (int a = 0; a < g.D; ++a) mm *= m1(d[a], h);
    for (int dir = 0; dir < g.D; ++dir) {
      double term = 1.0;
      for (int a = 0; a < g.D; ++a) term *= (a == dir) ? k1(d[a], h) : m1(d[a], h);
      kk += term;
    }
    // potential part: elements e_a in {gnode-1, gnode} (d=0), {gnode} (d=+1), {gnode-1} (d=-1)
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
            sum += eval_V(*vs, z) * shape;
          }
          double wvol = 1.0;
          for (int a = 0; a < g.D; ++a) wvol *= 0.5 * h;
          mv += wvol * sum;
        }
    tK[idx] = kk;
    tM[idx] = mm;
    tA[idx] = kk + mv;
  }
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

// y = T x over all interior unknowns of Omega_L; neighbours on the Dirichlet
// boundary are eliminated (skipped).  Work items are row segments of kBlock
// consecutive x1 positions (one grid line of dims 1..D-1 each), visited
// grid-stride by a fixed grid of kRedBlocks workgroups, so the index
// arithmetic is one division per segment.  Optional partial sums of x.y and of y.
template <int D>
__global__ void __launch_bounds__(kBlock) k_stencil(Geo g, const double* __restrict__ T,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y, int use_dot, Red dot,
                                                    int use_sum, Red sum) {
  double acc = 0.0, accs = 0.0;
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2];
  const long N01 = (long)N0 * N1;
  const int segs = (N0 + kBlock - 1) / kBlock;
  const long items = (long)segs * N1 * N2;
  const long tsize = g.tsize;
  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const int line = (int)(it / segs);
    const int i0 = (int)(it - (long)line * segs) * kBlock + threadIdx.x;
    if (i0 >= N0) continue;
    // line = i1r + N1 i2
    const int i2 = D == 3 ? (int)fdiv((unsigned)line, g.fN1) : 0;
    const int i1r = line - i2 * N1;
    const long k = i0 + (long)N0 * line;
    const int j0 = (int)((unsigned)(i0 + 1) - g.ne * fdiv((unsigned)(i0 + 1), g.fne));
    int j1 = i1r;
    if (g.isx[1]) j1 = (int)((unsigned)(i1r + 1) - g.ne * fdiv((unsigned)(i1r + 1), g.fne));
    const long tn = j0 + (long)g.P[0] * (j1 + (long)g.P[1] * i2);
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < (D == 2 ? 9 : 27); ++t) {
      const int d0 = t % 3 - 1, d1 = (t / 3) % 3 - 1, d2 = (D == 2) ? 0 : t / 9 - 1;
      const bool in = (i0 + d0 >= 0) && (i0 + d0 < N0) && (i1r + d1 >= 0) && (i1r + d1 < N1) &&
                      (D == 2 || ((i2 + d2 >= 0) && (i2 + d2 < N2)));
      if (in) s += T[t * tsize + tn] * x[k + d0 + (long)N0 * d1 + N01 * d2];
    }
    y[k] = s;
    acc += x[k] * s;
    accs += s;
  }
  if (use_dot) write_partial(acc, dot.part);
  if (use_sum) write_partial(accs, sum.part);
}

void launch_stencil(const ddeig_problem* P, const double* tab, const double* x, double* y,
                    Red* dot, Red* sum, hipStream_t s) {
  const long segs = (P->g.N[0] + kBlock - 1) / kBlock;
  const long items = segs * P->g.N[1] * P->g.N[2];
  const int blocks = (int)std::min<long>(items, kMaxRed);
  const Red none{nullptr, 0, nullptr};
  if (dot) dot->np = blocks;
  if (sum) sum->np = blocks;
  if (P->g.D == 2)
    hipLaunchKernelGGL(k_stencil<2>, dim3(blocks), dim3(kBlock), 0, s, P->g, tab, x, y,
                       dot ? 1 : 0, dot ? *dot : none, sum ? 1 : 0, sum ? *sum : none);
  else
    hipLaunchKernelGGL(k_stencil<3>, dim3(blocks), dim3(kBlock), 0, s, P->g, tab, x, y,
                       dot ? 1 : 0, dot ? *dot : none, sum ? 1 : 0, sum ? *sum : none);
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

// Hellmann-Feynman and adjoint forms for the derivatives of the eigenvalue,
// the shift and a shifted solve with respect to the Fourier parameters
// theta = (a_1..a_T, phi_1..phi_T) of the potential (beyond the paper).
//
// A = K + M_V (§2, eq:discrete-weak-form) is linear in V, so dA/dtheta_j is
// the mass matrix weighted by dV/dtheta_j with the same quadrature; for
//   V = sum_t a_t cos(arg_t) env,  arg_t = 2 pi k_t x1 (+ 2 pi m_t x2) + phi_t,
// (env = 1 + cy prod_j sin(pi y_j / ell) for SEP_FOURIER, 1 for FOURIER2)
//   dV/da_t = cos(arg_t) env,   dV/dphi_t = -a_t sin(arg_t) env.
// One kernel walks the elements of every job (a vector pair x, y on the grid
// or on the periodic cell of one problem) and, at each tensor 2-point Gauss
// point, interpolates x and y and adds w_q x_h y_h times each of the 2T
// derivative weights and times 1 (the mass form x^T M y), i.e. all 2T + 1
// forms x^T M_W y at once.  Jobs of many problems (a batch) share one
// launch: a block map assigns each workgroup to a job.  Per job and form the
// block partials are added in a fixed order by a second launch.
#include "k_common.h"

namespace ddeig {

constexpr int kGradTerms = 16;  // terms per launch (2 x 16 + 1 accumulators)

template <int CELL>
__device__ inline void grad_element(const GradJob& jb, long e, int t0, int nt, double* acc) {
  const double xi[2] = {0.5 * (1.0 - 0.57735026918962576450914878050196),
                        0.5 * (1.0 + 0.57735026918962576450914878050196)};
  const double two_pi = 6.283185307179586476925286766559;
  const double pi = 3.1415926535897932384626433832795;
  const Geo& g = jb.g;
  const VSpec& v = *jb.vs;
  const int D = g.D, nq = 1 << D;
  int nel[3] = {1, 1, 1};
  for (int a = 0; a < D; ++a) nel[a] = (CELL && g.isx[a]) ? g.ne : g.nel[a];
  int ee[3];
  ee[0] = (int)(e % nel[0]);
  ee[1] = (int)((e / nel[0]) % nel[1]);
  ee[2] = (int)(e / ((long)nel[0] * nel[1]));
  double xv[8], yv[8];
  for (int s = 0; s < nq; ++s) {
    long idx = 0, stride = 1;
    bool in = true;
    for (int a = 0; a < D; ++a) {
      const int node = ee[a] + ((s >> a) & 1);
      if (CELL && g.isx[a]) {
        idx += stride * (node % g.ne);
        stride *= g.ne;
      } else {
        const int u = node - 1;
        if (u < 0 || u >= g.N[a]) in = false;
        idx += stride * u;
        stride *= g.N[a];
      }
    }
    xv[s] = in ? jb.x[idx] : 0.0;
    yv[s] = in ? jb.y[idx] : 0.0;
  }
  double lo[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D; ++a) lo[a] = (double)(g.isx[a] ? ee[a] % g.ne : ee[a]) * g.h;
  double wvol = 1.0;
  for (int a = 0; a < D; ++a) wvol *= 0.5 * g.h;
  for (int qi = 0; qi < nq; ++qi) {
    double z[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) z[a] = lo[a] + g.h * xi[(qi >> a) & 1];
    double xh = 0.0, yh = 0.0;
    for (int s = 0; s < nq; ++s) {
      double N = 1.0;
      for (int a = 0; a < D; ++a) {
        const double t = xi[(qi >> a) & 1];
        N *= ((s >> a) & 1) ? t : 1.0 - t;
      }
      xh += N * xv[s];
      yh += N * yv[s];
    }
    const double w = wvol * xh * yh;
    double env = 1.0;
    if (v.kind == DDEIG_V_SEP_FOURIER) {
      double G = 1.0;
      for (int j = 0; j < v.q; ++j) G *= sin(pi * z[v.p + j] / v.ell);
      env = 1.0 + v.cy * G;
    }
    const double we = w * env;
#pragma unroll
    for (int t = 0; t < kGradTerms; ++t) {
      if (t < nt) {
        const int tt = t0 + t;
        const double arg = v.kind == DDEIG_V_FOURIER2
                               ? two_pi * (v.k[tt] * z[0] + v.m[tt] * z[1]) + v.phi[tt]
                               : two_pi * v.k[tt] * z[0] + v.phi[tt];
        double sn, cs;
        sincos(arg, &sn, &cs);
        acc[t] += we * cs;
        acc[kGradTerms + t] -= we * v.a[tt] * sn;
      }
    }
    acc[2 * kGradTerms] += w;
  }
}

// Forms of terms [t0, t0 + nt) (and the mass form) of every job; block b of the
// launch works for job map[b].x as its block map[b].y.  Partials:
// part[jb.part0 + f * jb.nblk + block], f = term (a_t), T + term (phi_t), 2T (mass).
__global__ void __launch_bounds__(kBlock) k_grad_forms(const GradJob* __restrict__ jobs,
                                                       const int2* __restrict__ map, int T, int t0,
                                                       int nt, int with_mass,
                                                       double* __restrict__ part) {
  const int2 jm = map[blockIdx.x];
  const GradJob jb = jobs[jm.x];
  double acc[2 * kGradTerms + 1];
#pragma unroll
  for (int f = 0; f < 2 * kGradTerms + 1; ++f) acc[f] = 0.0;
  for (long e = jm.y * (long)kBlock + threadIdx.x; e < jb.nelem; e += (long)jb.nblk * kBlock) {
    if (jb.cell) grad_element<1>(jb, e, t0, nt, acc);
    else grad_element<0>(jb, e, t0, nt, acc);
  }
  double* p = part + jb.part0;
#pragma unroll
  for (int t = 0; t < kGradTerms; ++t) {
    if (t < nt) {
      const double sa = block_sum(acc[t]);
      const double sp = block_sum(acc[kGradTerms + t]);
      if (threadIdx.x == 0) {
        p[(long)(t0 + t) * jb.nblk + jm.y] = sa;
        p[(long)(T + t0 + t) * jb.nblk + jm.y] = sp;
      }
    }
  }
  if (with_mass) {
    const double sm = block_sum(acc[2 * kGradTerms]);
    if (threadIdx.x == 0) p[(long)(2 * T) * jb.nblk + jm.y] = sm;
  }
}

// out[j * nf + f] = sum of the block partials of form f of job j, in block order.
__global__ void k_grad_finish(const GradJob* __restrict__ jobs, int nf, const double* __restrict__ part,
                              double* __restrict__ out) {
  const int j = blockIdx.x / nf, f = blockIdx.x % nf;
  const GradJob jb = jobs[j];
  const double v = sum_partials(part + jb.part0 + (long)f * jb.nblk, jb.nblk);
  if (threadIdx.x == 0) out[(long)j * nf + f] = v;
}

int grad_blocks(long nelem) {
  return (int)std::max<long>(1, std::min<long>(256, (nelem + kBlock - 1) / kBlock));
}

void launch_grad_forms(const GradJob* dJobs, const int2* dMap, int nblocks, int njobs, int T,
                       double* part, double* out, hipStream_t s) {
  for (int t0 = 0; t0 < T; t0 += kGradTerms) {
    const int nt = std::min(kGradTerms, T - t0);
    hipLaunchKernelGGL(k_grad_forms, dim3(nblocks), dim3(kBlock), 0, s, dJobs, dMap, T, t0, nt,
                       t0 == 0 ? 1 : 0, part);
  }
  hipLaunchKernelGGL(k_grad_finish, dim3(njobs * (2 * T + 1)), dim3(kBlock), 0, s, dJobs,
                     2 * T + 1, part, out);
}

}  // namespace ddeig

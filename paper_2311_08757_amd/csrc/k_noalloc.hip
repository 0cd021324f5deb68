// The potential-weighted form x^T M_W y without any device allocation, for
// callers that cannot allocate (code under graph capture, tight serving loops).
//
// M_W is the mass matrix weighted by W with the quadrature of A = K + M_V (§2,
// eq:discrete-weak-form: tensor 2-point Gauss-Legendre per element, W at
// cell-local x).  Instead of a stencil table of M_W and an intermediate
// vector M_W y, one kernel walks the elements: at each quadrature point it
// interpolates x and y from the element's 2^D nodes (zero at Dirichlet nodes)
// and adds w_q W(z_q) x_h(z_q) y_h(z_q), which is x^T M_W y summed element by
// element.  Its only device memory besides x and y is the file-scope array
// `scratch` (1 MiB, one copy per GPU, held until the process ends): the block
// partial sums, the result, the copy of W's description and, for a tabulated
// W, its quadrature-point values.  Every call rewrites what it reads, so
// nothing needs clearing; two calls that overlap on one GPU race on it.
#include <mutex>

#include "k_common.h"

namespace ddeig {

constexpr long kNaDoubles = 131072;   // 1 MiB
constexpr int kNaParts = 1024;        // block partials [0, 1024), result at 1024
constexpr long kNaSpecOff = 1040;     // the copy of W's description (< 8 KiB)
constexpr long kNaTabOff = 2048;      // QUAD_TABLE values
constexpr long kNaTabMax = kNaDoubles - kNaTabOff;
static_assert(sizeof(VSpec) <= (kNaTabOff - kNaSpecOff) * sizeof(double), "VSpec fits");

static __device__ __align__(256) double scratch[kNaDoubles];

namespace {
constexpr int kNaMaxDev = 64;
std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDev] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (called by ddeig_assemble with the problem's device current).
hipError_t noalloc_init(int dev) {
  if (dev < 0 || dev >= kNaMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (g_na_ptr[dev] != nullptr) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_na_ptr[dev] = static_cast<double*>(p);
  return hipSuccess;
}

static double* noalloc_ptr(int dev) {
  if (dev < 0 || dev >= kNaMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(g_na_mu);
  return g_na_ptr[dev];
}

// x^T M_W y over the elements of the grid (CELL = 0) or of the periodic cell
// (CELL = 1); one partial per block into part.
template <int CELL>
__global__ void __launch_bounds__(kBlock) k_na_form(Geo g, const VSpec* __restrict__ ws,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ y, long nelem,
                                                    double* __restrict__ part) {
  const double xi[2] = {0.5 * (1.0 - 0.57735026918962576450914878050196),
                        0.5 * (1.0 + 0.57735026918962576450914878050196)};
  const VSpec& v = *ws;
  const int D = g.D, nq = 1 << D;
  int nel[3] = {1, 1, 1};  // elements per dim of the walked mesh
  for (int a = 0; a < D; ++a) nel[a] = (CELL && g.isx[a]) ? g.ne : g.nel[a];
  double acc = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nelem;
       e += (long)gridDim.x * blockDim.x) {
    int ee[3];
    ee[0] = (int)(e % nel[0]);
    ee[1] = (int)((e / nel[0]) % nel[1]);
    ee[2] = (int)(e / ((long)nel[0] * nel[1]));
    // node values of the element (s = sum_a s_a 2^a), zero at Dirichlet nodes
    double xv[8], yv[8];
    for (int s = 0; s < nq; ++s) {
      long idx = 0, stride = 1;
      bool in = true;
      for (int a = 0; a < D; ++a) {
        const int node = ee[a] + ((s >> a) & 1);
        int u;
        if (CELL && g.isx[a]) {
          u = node % g.ne;
          idx += stride * u;
          stride *= g.ne;
        } else {
          u = node - 1;
          if (u < 0 || u >= g.N[a]) in = false;
          idx += stride * u;
          stride *= g.N[a];
        }
      }
      xv[s] = in ? x[idx] : 0.0;
      yv[s] = in ? y[idx] : 0.0;
    }
    double lo[3];
    long tab0 = 0;
    {
      long stride = nq;
      for (int a = 0; a < D; ++a) {
        const int el = g.isx[a] ? ee[a] % g.ne : ee[a];
        lo[a] = (double)el * g.h;
        tab0 += stride * el;
        stride *= g.isx[a] ? g.ne : g.nel[a];
      }
    }
    double sum = 0.0;
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
      const double wq = v.kind == DDEIG_V_QUAD_TABLE ? v.table[tab0 + qi] : eval_V(v, z);
      sum += wq * xh * yh;
    }
    double wvol = 1.0;
    for (int a = 0; a < D; ++a) wvol *= 0.5 * g.h;
    acc += wvol * sum;
  }
  write_partial(acc, part);
}

__global__ void k_na_finish(double* __restrict__ part, int np) {
  const double v = sum_partials(part, np);
  if (threadIdx.x == 0) part[kNaParts] = v;
}

// The body of ddeig_potential_form_noalloc after its argument checks (api.hip):
// copies W's description (and table) into the scratch, walks the elements,
// adds the block partials in order and returns the form in *out (synchronises).
ddeig_status noalloc_form_checked(ddeig_problem* P, int space, const VSpec& wspec, const double* table,
                                  long table_len, const double* x, const double* y, double* out,
                                  std::string& err) {
  double* sp = noalloc_ptr(P->device);
  if (sp == nullptr) {
    err = "the no-allocation scratch of this device was not set up";
    return DDEIG_EHIP;
  }
  if (table != nullptr && table_len > kNaTabMax) {
    err = "the weight table has " + std::to_string(table_len) + " values; the no-allocation " +
          "scratch holds at most " + std::to_string(kNaTabMax);
    return DDEIG_EINVAL;
  }
  const hipStream_t s = P->stream;
  VSpec ws = wspec;
  if (table != nullptr) {
    check_hip(hipMemcpyAsync(sp + kNaTabOff, table, sizeof(double) * table_len,
                             hipMemcpyHostToDevice, s), "copy weight table");
    ws.table = sp + kNaTabOff;
  }
  check_hip(hipMemcpyAsync(sp + kNaSpecOff, &ws, sizeof(VSpec), hipMemcpyHostToDevice, s),
            "copy W");
  const Geo& g = P->g;
  long nelem = 1;
  for (int a = 0; a < g.D; ++a) nelem *= (space == 1 && g.isx[a]) ? g.ne : g.nel[a];
  const int np = (int)std::min<long>(kNaParts, (nelem + kBlock - 1) / kBlock);
  const VSpec* dws = reinterpret_cast<const VSpec*>(sp + kNaSpecOff);
  if (space == 0)
    hipLaunchKernelGGL(k_na_form<0>, dim3(np), dim3(kBlock), 0, s, g, dws, x, y, nelem, sp);
  else
    hipLaunchKernelGGL(k_na_form<1>, dim3(np), dim3(kBlock), 0, s, g, dws, x, y, nelem, sp);
  hipLaunchKernelGGL(k_na_finish, dim3(1), dim3(kBlock), 0, s, sp, np);
  check_hip(hipGetLastError(), "potential form (no allocation)");
  check_hip(hipMemcpyAsync(out, sp + kNaParts, sizeof(double), hipMemcpyDeviceToHost, s),
            "copy form");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  return DDEIG_OK;
}

}  // namespace ddeig

// Host side of libddeig: argument validation, decomposition bookkeeping,
// device memory, and the drivers of the cell problem, PCG and inverse
// iteration.  Every call returns a ddeig_status; HIP failures and
// allocation failures are turned into status codes here.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "k_common.h"

using namespace ddeig;

namespace {

thread_local std::string g_last_error;

struct Failure {
  ddeig_status status;
  std::string msg;
};

ddeig_status set_error(ddeig_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

template <typename T>
T* dalloc(ddeig_problem* P, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Failure{DDEIG_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
  }
  P->allocs.push_back(p);
  return static_cast<T*>(p);
}

void dfree(ddeig_problem* P, void* p) {
  if (!p) return;
  auto it = std::find(P->allocs.begin(), P->allocs.end(), p);
  if (it != P->allocs.end()) P->allocs.erase(it);
  (void)hipFree(p);
}

void sync(ddeig_problem* P) { check_hip(hipStreamSynchronize(P->stream), "hipStreamSynchronize"); }

// A device buffer of at least `need` elements, replacing a smaller one (owned
// through `allocs`).
template <typename T>
T* grow(std::vector<void*>& allocs, T* old, long& cap, long need) {
  if (old != nullptr && cap >= need) return old;
  if (old != nullptr) {
    auto it = std::find(allocs.begin(), allocs.end(), (void*)old);
    if (it != allocs.end()) allocs.erase(it);
    (void)hipFree(old);
    cap = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * (size_t)std::max<long>(need, 1)) != hipSuccess) {
    (void)hipGetLastError();
    throw Failure{DDEIG_ENOMEM, "hipMalloc of the derivative-form buffers failed"};
  }
  allocs.push_back(p);
  cap = need;
  return static_cast<T*>(p);
}

// All 2T + 1 forms x^T M_W y (W = dV/da_t, dV/dphi_t, 1) of every job in one
// grouped launch; out receives njobs x (2T + 1) values.  Synchronises s.
void grad_run(std::vector<void*>& allocs, GradBuf& gb, std::vector<GradJob>& jobs, int T,
              hipStream_t s, std::vector<double>& out) {
  const int nf = 2 * T + 1;
  std::vector<int2> map;
  long part = 0;
  for (int j = 0; j < (int)jobs.size(); ++j) {
    jobs[j].nblk = grad_blocks(jobs[j].nelem);
    jobs[j].part0 = part;
    part += (long)nf * jobs[j].nblk;
    for (int b = 0; b < jobs[j].nblk; ++b) map.push_back(make_int2(j, b));
  }
  gb.jobs = grow(allocs, gb.jobs, gb.cap_jobs, (long)jobs.size());
  gb.map = grow(allocs, gb.map, gb.cap_map, (long)map.size());
  gb.part = grow(allocs, gb.part, gb.cap_part, part);
  gb.out = grow(allocs, gb.out, gb.cap_out, (long)jobs.size() * nf);
  check_hip(hipMemcpyAsync(gb.jobs, jobs.data(), sizeof(GradJob) * jobs.size(),
                           hipMemcpyHostToDevice, s), "copy derivative jobs");
  check_hip(hipMemcpyAsync(gb.map, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice, s),
            "copy block map");
  launch_grad_forms(gb.jobs, gb.map, (int)map.size(), (int)jobs.size(), T, gb.part, gb.out, s);
  check_hip(hipGetLastError(), "derivative forms");
  out.assign(jobs.size() * (size_t)nf, 0.0);
  check_hip(hipMemcpyAsync(out.data(), gb.out, sizeof(double) * out.size(), hipMemcpyDeviceToHost, s),
            "copy forms");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// The job of the pair (x, y) of problem P on its grid (cell = 0) or periodic cell.
GradJob grad_job(const ddeig_problem* P, const double* x, const double* y, int cell) {
  GradJob jb{};
  jb.g = P->g;
  jb.vs = P->dVS;
  jb.x = x;
  jb.y = y;
  jb.cell = cell;
  long ne = 1;
  for (int a = 0; a < P->g.D; ++a) ne *= (cell && P->g.isx[a]) ? P->g.ne : P->g.nel[a];
  jb.nelem = ne;
  return jb;
}

// The number of Fourier parameters of the problem's potential (2T), or an error.
ddeig_status grad_params(const ddeig_problem* P, int ngrad, int& T) {
  if (P->vs.kind != DDEIG_V_SEP_FOURIER && P->vs.kind != DDEIG_V_FOURIER2)
    return set_error(DDEIG_EINVAL, "derivatives need a SEP_FOURIER or FOURIER2 potential");
  T = P->vs.nterms;
  if (ngrad != 2 * T)
    return set_error(DDEIG_EINVAL, "ngrad must be 2 nterms = " + std::to_string(2 * T));
  return DDEIG_OK;
}

void check_launch(const char* what) { check_hip(hipGetLastError(), what); }

Red slot(ddeig_problem* P, int i) {
  return Red{P->red_part + (long)i * kMaxRed, 0, P->red_val + i};
}

double host_sum(ddeig_problem* P, Red r) {
  launch_finish_sum(r, P->stream);
  double v = 0.0;
  check_hip(hipMemcpyAsync(&v, r.val, sizeof(double), hipMemcpyDeviceToHost, P->stream),
            "copy scalar");
  sync(P);
  return v;
}

// The cell box: whole unit cell, periodic in x (origin -1 so that the node
// index equals the cell index), all fixed-direction unknowns.
Box cell_box(const Geo& g) {
  Box b;
  for (int a = 0; a < 3; ++a) {
    if (a >= g.D) {
      b.o[a] = 0; b.m[a] = 1; b.per[a] = 0;
    } else if (g.isx[a]) {
      b.o[a] = -1; b.m[a] = g.ne; b.per[a] = 1;
    } else {
      b.o[a] = 0; b.m[a] = g.N[a]; b.per[a] = 0;
    }
  }
  b.b = 1;
  for (int a = 0; a < g.D - 1; ++a) b.b *= b.m[a];
  b.nch = b.m[g.D - 1];
  return b;
}

// Smallest generalised eigenvalue of the 1-D Dirichlet linear-element pair
// with nel elements: mu(theta) = (6/h^2)(1 - cos theta)/(2 + cos theta), theta = pi / nel.
double mu_min(int nel, double h) {
  const double th = M_PI / nel;
  return 6.0 / (h * h) * (1.0 - std::cos(th)) / (2.0 + std::cos(th));
}

// min of V over the 2-point Gauss points of the cell elements
double cell_vmin(const ddeig_problem* P) {
  const Geo& g = P->g;
  if (P->vs.kind == DDEIG_V_QUAD_TABLE)
    return *std::min_element(P->vtab_host.begin(), P->vtab_host.end());
  const double xs[2] = {0.5 * (1.0 - 1.0 / std::sqrt(3.0)), 0.5 * (1.0 + 1.0 / std::sqrt(3.0))};
  int ecount[3] = {1, 1, 1};
  for (int a = 0; a < g.D; ++a) ecount[a] = g.isx[a] ? g.ne : g.nel[a];
  double vmin = INFINITY;
  for (int e2 = 0; e2 < ecount[2]; ++e2)
    for (int e1 = 0; e1 < ecount[1]; ++e1)
      for (int e0 = 0; e0 < ecount[0]; ++e0) {
        const int ee[3] = {e0, e1, e2};
        for (int qi = 0; qi < (1 << g.D); ++qi) {
          double z[3] = {0, 0, 0};
          for (int a = 0; a < g.D; ++a) z[a] = (ee[a] + xs[(qi >> a) & 1]) * g.h;
          vmin = std::min(vmin, eval_V(P->vs, z));
        }
      }
  return vmin;
}

void factor_types(ddeig_problem* P) {
  if (P->opt.local_prec >= 2) {
    // dense local solves: FP64 block-chain factors of the unclipped box, its
    // inverse from the chain solves of the identity columns, the bf16 (hi /
    // lo) split, then for every clipped class (B~_TT)^{-1} from the rounded
    // inverse (FP64 Gauss-Jordan, symmetrised) and G = B~_ST (B~_TT)^{-1}
    ddeig::DenseHost& H = P->dh;
    chain_factor(P, H.box, P->tabAs, H.W, P->stream);
    check_launch("local factorisation");
    double* Ainv = dalloc<double>(P, (size_t)H.m * H.m);
    launch_identity(Ainv, H.m, P->stream);
    launch_chain_solve_box(P, H.box, P->tabAs, H.W, Ainv, H.m, P->stream);
    launch_split_inverse(Ainv, H.m, H.ld, H.Ah, H.Al, P->stream);
    check_launch("dense inverse");
    sync(P);
    dfree(P, Ainv);
    for (const auto& E : P->emb) {
      double* C = dalloc<double>(P, (size_t)E.nT * E.nT);
      launch_embed_gather(P, E, C, P->stream);
      launch_gj_invert(P, C, E.nT, P->stream);
      launch_symmetrise(C, E.nT, P->stream);
      launch_embed_gmat(P, E, C, const_cast<float*>(E.G), P->stream);
      check_launch("clipped-class corrections");
      sync(P);
      dfree(P, C);
    }
    return;
  }
  for (auto& t : P->types) {
    chain_factor(P, t.box, P->tabAs, t.W, P->stream);
    if (P->opt.local_prec == 1) {
      if (P->chain_mfma)
        launch_pad_float(t.W, t.W32, (long)t.box.nch * t.box.b, t.box.b, (t.box.b + 3) / 4 * 4,
                         P->stream);
      else
        launch_to_float(t.W, t.W32, (long)t.box.nch * t.box.b * t.box.b, P->stream);
    }
  }
  check_launch("local factorisation");
}

int read_flag(ddeig_problem* P) {
  int f = 0;
  check_hip(hipMemcpyAsync(&f, P->flag, sizeof(int), hipMemcpyDeviceToHost, P->stream), "flag");
  sync(P);
  return f;
}

void clear_flag(ddeig_problem* P) {
  check_hip(hipMemsetAsync(P->flag, 0, sizeof(int), P->stream), "memset flag");
}

void clear_graphs(ddeig_problem* P) {
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  for (auto& kv : P->gm_graphs) (void)hipGraphExecDestroy(kv.second);
  P->gm_graphs.clear();
}

// Captures the launches of `body` on the problem's capture stream into a HIP
// graph and instantiates it.
template <typename F>
hipGraphExec_t capture_graph(ddeig_problem* P, F&& body) {
  hipGraph_t gr = nullptr;
  hipGraphExec_t ge = nullptr;
  check_hip(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    body(P->cap);
  } catch (...) {
    (void)hipStreamEndCapture(P->cap, &gr);
    if (gr) (void)hipGraphDestroy(gr);
    throw;
  }
  check_hip(hipStreamEndCapture(P->cap, &gr), "end capture");
  const hipError_t e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  check_hip(e, "instantiate graph");
  return ge;
}

// sigma-dependent set-up: shifted table, local factors, coarse matrix.
ddeig_status finish_shift(ddeig_problem* P) {
  clear_graphs(P);
  launch_shift_table(P, P->stream);
  clear_flag(P);
  factor_types(P);
  if (read_flag(P)) return set_error(DDEIG_ENOTSPD, "a local matrix A_sigma,i is not positive definite");
  if (P->opt.coarse) {
    launch_coarse_phi(P, P->stream);
    build_coarse_matrix(P, P->A0inv, P->stream);
    launch_gj_invert(P, P->A0inv, P->nsub, P->stream);
    launch_symmetrise(P->A0inv, P->nsub, P->stream);
    check_launch("coarse set-up");
    if (read_flag(P)) return set_error(DDEIG_ENOTSPD, "the coarse matrix A_sigma,0 is not positive definite");
  }
  P->shifted = 1;
  return DDEIG_OK;
}

// Parts of a Schwarz preconditioner (kind argument of precond_apply): the
// local solves, the coarse correction, and the partition-of-unity weighting of
// the local solutions (restricted additive Schwarz).
constexpr int kPrecLocal = 1, kPrecCoarse = 2, kPrecRas = 4;

int prec_flags(int kind) {
  switch (kind) {
    case DDEIG_PREC_AS1: return kPrecLocal;
    case DDEIG_PREC_AS2: return kPrecLocal | kPrecCoarse;
    case DDEIG_PREC_RAS1: return kPrecLocal | kPrecRas;
    case DDEIG_PREC_RAS2: return kPrecLocal | kPrecCoarse | kPrecRas;
    case DDEIG_PREC_COARSE: return kPrecCoarse;
    default: return -1;
  }
}

// Automatic fallback when CG breaks down with r.z <= 0 under the dense
// reduced-precision local solves (the rounded inverse made M^{-1} indefinite):
// the problem switches to FP32 block-chain local solves (FP64 factors of
// every class, rounded to FP32) for the rest of its life, and the caller
// repeats the solve.  2-D problems only (their chain solves need no further
// set-up); returns false where no fallback exists.
bool fallback_fp32(ddeig_problem* P) {
  if (P->opt.local_prec < 2 || P->g.D != 2) return false;
  const hipStream_t s = P->stream;
  std::vector<TypeDev> tdev(P->types.size());
  check_hip(hipMemcpy(tdev.data(), P->dTypes, sizeof(TypeDev) * tdev.size(), hipMemcpyDeviceToHost),
            "read classes");
  for (size_t t = 0; t < P->types.size(); ++t) {
    auto& T = P->types[t];
    const long mm = (long)T.box.nch * T.box.b;
    T.W = dalloc<double>(P, (size_t)T.box.nch * T.box.b * T.box.b);
    T.W32 = dalloc<float>(P, (size_t)T.box.nch * T.box.b * T.box.b);
    dfree(P, T.batch);
    T.batch = dalloc<double>(P, (size_t)T.nmem * mm);
    TypeDev& d = tdev[t];
    for (int a = 0; a < 3; ++a) {
      d.hm[a] = T.box.m[a];
      d.off[a] = 0;
    }
    d.dense = 0;
    d.W = T.W;
    d.W32 = T.W32;
    d.batch = T.batch;
    d.tbatch = nullptr;
    d.ld = 0;
    d.ksplit = 0;
    d.Rh = d.Rl = nullptr;
    d.Z = nullptr;
    d.zsplit = 0;
    d.ldw = T.box.b;
  }
  std::vector<SubTS> ts(P->nsub);
  for (int sid = 0; sid < P->nsub; ++sid) ts[sid] = SubTS{P->subs[sid].type, P->subs[sid].slot};
  check_hip(hipMemcpy(P->dTypes, tdev.data(), sizeof(TypeDev) * tdev.size(), hipMemcpyHostToDevice),
            "write classes");
  check_hip(hipMemcpy(P->dSubTS, ts.data(), sizeof(SubTS) * ts.size(), hipMemcpyHostToDevice),
            "write subdomain table");
  P->opt.local_prec = 1;
  clear_graphs(P);
  clear_flag(P);
  for (auto& T : P->types) {
    chain_factor(P, T.box, P->tabAs, T.W, s);
    launch_to_float(T.W, T.W32, (long)T.box.nch * T.box.b * T.box.b, s);
  }
  check_launch("fallback factorisation");
  if (read_flag(P)) throw Failure{DDEIG_ENOTSPD, "a local matrix A_sigma,i is not positive definite"};
  ++P->fallbacks;
  return true;
}

// restrict -> {local solves (+ clipped-class correction) | coarse solve on the
// second stream} -> extend.  xr (nullable) fuses the CG update of x and r into the
// restriction (partials of ||r||^2 into *rr); chk (nullable) folds the PCG
// stopping test into the extension.  flags (kPrec*; -1: the problem's additive
// Schwarz preconditioner) selects the parts; the coarse correction alone runs
// on the library stream.
void precond_apply(ddeig_problem* P, double* r, double* z, Red* dot, PcgState* st,
                   const XrArgs* xr = nullptr, Red* rr = nullptr, const CheckArgs* chk = nullptr,
                   hipStream_t ms = nullptr, int flags = -1) {
  const hipStream_t s = ms ? ms : P->stream;
  if (flags < 0) flags = kPrecLocal | (P->opt.coarse ? kPrecCoarse : 0);
  const int coarse = (flags & kPrecCoarse) ? 1 : 0;
  if (!(flags & kPrecLocal)) {
    launch_coarse_rhs(P, r, st, s);
    launch_coarse_solve(P, st, s);
    launch_coarse_field(P, st, s);
    launch_coarse_extend(P, r, z, dot, st, s);
    return;
  }
  XrArgs xoff{};
  xoff.on = 0;
  CheckArgs coff{};
  coff.on = 0;
  launch_restrict(P, r, st, xr ? *xr : xoff, rr, s);
  if (coarse && fused_coarse(P)) {
    // one stream: R_0 r rides in the GEMM launch, A_0^{-1} c in the
    // clipped-class correction launch, the coarse field in the extension
    launch_local_solves(P, st, s, r);
    launch_embed_fix(P, st, s, true);
    CheckArgs c = chk ? *chk : coff;
    if (chk && rr) c.rr = *rr;
    launch_extend(P, r, z, 1, dot, st, c, s, (flags & kPrecRas) ? 1 : 0, 1);
    return;
  }
  const bool side = coarse;
  if (side) {
    check_hip(hipEventRecord(P->ev_fork, s), "record fork");
    check_hip(hipStreamWaitEvent(P->aux, P->ev_fork, 0), "wait fork");
  }
  launch_local_solves(P, st, s);
  if (P->opt.local_prec >= 2) launch_embed_fix(P, st, s);
  if (coarse) {
    launch_coarse_rhs(P, r, st, P->aux);
    launch_coarse_solve(P, st, P->aux);
    if (P->opt.local_prec >= 2) launch_coarse_field(P, st, P->aux);
  }
  if (side) {
    check_hip(hipEventRecord(P->ev_join, P->aux), "record join");
    check_hip(hipStreamWaitEvent(s, P->ev_join, 0), "wait join");
  }

  CheckArgs c = chk ? *chk : coff;
  if (chk && rr) c.rr = *rr;
  launch_extend(P, r, z, coarse, dot, st, c, s, (flags & kPrecRas) ? 1 : 0);
}

struct PcgOut {
  int iters = 0;
  double relres = 0.0;
  int done = 0;
};

// PCG on A_sigma x = b (x holds x0).  One iteration is four kernels on the
// library stream: the stencil with the direction update, the restriction with
// the x / r update, the local solves and the extension with the stopping test
// (plus the coarse solve on the second stream).  `batch` iterations are queued
// between host checks of the device state.
PcgOut pcg_run(ddeig_problem* P, const double* b, double* x, double rtol, int maxit) {
  const hipStream_t s = P->stream;
  const int batch = P->opt.batch_iters > 0 ? P->opt.batch_iters : 8;
  Red g = slot(P, 0), rr = slot(P, 1), rz = slot(P, 2);
  launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
  launch_resid_init(P, b, P->q, P->r, rr, s);
  // a test override makes the breakdown test of a reduced-precision solve fire
  double rz_floor = 0.0;
  if (P->force_rz > 0 && P->opt.local_prec >= 2) {
    rz_floor = INFINITY;
    --P->force_rz;
  }
  launch_pcg_init(P, rtol, rr, s, rz_floor);
  precond_apply(P, P->r, P->z, &rz, P->st);
  check_launch("pcg start");
  PcgState hs{};
  int k = 0;
  if (maxit <= 0) {
    check_hip(hipMemcpyAsync(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s), "state");
    sync(P);
  }
  // iteration k on stream ms
  auto iteration = [&](int kk, hipStream_t ms) {
    double* pold = P->pp[(kk - 1) & 1];
    double* pnew = P->pp[kk & 1];
    const DirArgs dir{P->st, kk, rz};
    launch_stencil_dir(P, P->z, pold, pnew, P->q, dir, g, ms);
    const XrArgs xr{1, kk, g, x, pnew, P->q};
    const CheckArgs chk{1, kk, maxit, P->hist_cap, rr, P->hist};
    precond_apply(P, P->r, P->z, &rz, P->st, &xr, &rr, &chk, ms);
  };
  // queues the block of iterations k0..kend and a copy of the CG state behind
  // it (into pinned host slot `sl`, signalled by ev_state[sl])
  auto submit = [&](int k0, int kend, int sl) {
    if (P->opt.graphs) {
      // the block, captured once per (k0, kend, maxit, x) on the problem's own
      // capture stream and replayed on the library stream
      const auto key = std::make_tuple(k0, kend, maxit, (const void*)x);
      auto it = P->graphs.find(key);
      if (it == P->graphs.end()) {
        if (P->graphs.size() >= 1024) {
          for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
          P->graphs.clear();
        }
        hipGraph_t gr = nullptr;
        hipGraphExec_t ge = nullptr;
        check_hip(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
          for (int kk = k0; kk <= kend; ++kk) iteration(kk, P->cap);
        } catch (...) {
          (void)hipStreamEndCapture(P->cap, &gr);
          if (gr) (void)hipGraphDestroy(gr);
          throw;
        }
        check_hip(hipStreamEndCapture(P->cap, &gr), "end capture");
        const hipError_t e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        check_hip(e, "instantiate graph");
        it = P->graphs.emplace(key, ge).first;
      }
      check_hip(hipGraphLaunch(it->second, s), "launch graph");
    } else {
      for (int kk = k0; kk <= kend; ++kk) iteration(kk, s);
    }
    check_launch("pcg iteration");
    check_hip(hipMemcpyAsync(&P->hst[sl], P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s),
              "state");
    check_hip(hipEventRecord(P->ev_state[sl], s), "record state");
  };
  // One block runs ahead: while the host waits for the state after block j,
  // block j + 1 is already queued, so the device does not idle during the
  // check.  Once CG has stopped, the block run ahead finds the done flag and
  // its kernels return at once.
  if (k < maxit) {
    const int kend = std::min(maxit, k + batch);
    submit(k + 1, kend, 0);
    k = kend;
    int cur = 0;
    for (;;) {
      bool ahead = false;
      if (k < maxit) {
        const int kend2 = std::min(maxit, k + batch);
        submit(k + 1, kend2, 1 - cur);
        k = kend2;
        ahead = true;
      }
      check_hip(hipEventSynchronize(P->ev_state[cur]), "state");
      hs = P->hst[cur];
      if (hs.done || !ahead) break;
      cur = 1 - cur;
    }
  }
  PcgOut o;
  o.iters = hs.iters;
  o.relres = hs.relres;
  o.done = hs.done;
  if (maxit <= 0 && hs.done == 0) o.done = 4;
  return o;
}

// Stationary restricted additive Schwarz for A_sigma x = b (x holds x0):
// levels 1: x_{k+1} = x_k + M_RAS,1^{-1} r_k (eq:stationary-ras); levels 2:
// the same half step followed by the coarse correction of the new residual
// (eq:two-level-stationary-ras-mult-cc).  Each half step: the preconditioner
// part into z, x += z, then the residual r = b - A_sigma x afresh with the
// partials of ||r||^2 (no recurrence, so no drift over many steps); the
// stopping test ||r_k|| <= rtol ||r_0|| closes every step.
PcgOut sras_run(ddeig_problem* P, int levels, const double* b, double* x, double rtol,
                int maxit) {
  const hipStream_t s = P->stream;
  const int batch = P->opt.batch_iters > 0 ? P->opt.batch_iters : 8;
  Red rr = slot(P, 1);
  launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
  launch_resid_init(P, b, P->q, P->r, rr, s);
  launch_pcg_init(P, rtol, rr, s);
  check_launch("stationary RAS start");
  PcgState hs{};
  check_hip(hipMemcpyAsync(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s), "state");
  sync(P);
  int k = 0;
  while (k < maxit && !hs.done) {
    const int kend = std::min(maxit, k + batch);
    for (int kk = k + 1; kk <= kend; ++kk) {
      precond_apply(P, P->r, P->z, nullptr, P->st, nullptr, nullptr, nullptr, s,
                    kPrecLocal | kPrecRas);
      launch_sr_update(P, P->z, x, s);
      launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
      launch_resid_init(P, b, P->q, P->r, rr, s);
      if (levels == 2) {
        precond_apply(P, P->r, P->z, nullptr, P->st, nullptr, nullptr, nullptr, s, kPrecCoarse);
        launch_sr_update(P, P->z, x, s);
        launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
        launch_resid_init(P, b, P->q, P->r, rr, s);
      }
      launch_sr_check(P, rr, kk, maxit, s);
    }
    k = kend;
    check_launch("stationary RAS step");
    check_hip(hipMemcpyAsync(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s), "state");
    sync(P);
  }
  PcgOut o;
  o.iters = hs.iters;
  o.relres = hs.relres;
  o.done = hs.done ? hs.done : 4;
  return o;
}

// GMRES work space for restart length m: V (m + 1 vectors), Z (m vectors), w,
// the dot partials ((2m + 3) rows x blocks) and their sums d, H ((m + 1) x m),
// rotations cs, sn (m), g (m + 1), the first-pass scales c (m + 1), scalars and y (m).
struct GmWs {
  double *V, *Z, *w, *part, *d, *H, *cs, *sn, *g, *cv, *gm, *y;
  long ldv;
};

GmWs gm_workspace(ddeig_problem* P, int m) {
  const long n = P->g.n;
  const long ldv = gm_stride(n);
  const long nb = gm_blocks(n);
  long off = 0;
  auto take = [&](long cnt) {
    const long o = off;
    off += cnt;
    return o;
  };
  const long oV = take((long)(m + 1) * ldv), oZ = take((long)m * ldv), oW = take(ldv);
  const long oP = take((long)(2 * m + 3) * nb), oD = take(2 * m + 3);
  const long oH = take((long)(m + 1) * m), oC = take(m), oS = take(m), oG = take(m + 1);
  const long oCv = take(m + 1), oM = take(8), oY = take(m);
  if (m > P->gm_cap || ldv != P->gm_ldv || !P->gmws) {
    for (auto& kv : P->gm_graphs) (void)hipGraphExecDestroy(kv.second);
    P->gm_graphs.clear();
    dfree(P, P->gmws);
    P->gmws = nullptr;
    P->gm_cap = 0;
    P->gmws = dalloc<double>(P, (size_t)off);
    P->gm_cap = m;
    P->gm_ldv = ldv;
    // the basis kernels read every vector up to the stride: the entries beyond
    // n stay zero (nothing writes them)
    check_hip(hipMemsetAsync(P->gmws, 0, sizeof(double) * (size_t)off, P->stream), "clear");
  }
  double* b = P->gmws;
  return GmWs{b + oV, b + oZ, b + oW, b + oP, b + oD, b + oH, b + oC, b + oS, b + oG, b + oCv,
              b + oM, b + oY, ldv};
}

// GMRES for A_sigma x = b (x holds x0) with right preconditioning by the
// Schwarz preconditioner of `flags`, restarted every m steps; one step is
// described in k_krylov.hip.  A cycle runs steps j = 0..jmax, jmax =
// min(m, maxit - k0): step j applies the preconditioner and A_sigma to u_j
// (not for j = jmax, which only finishes the last column) and completes
// Hessenberg column j - 1, i.e. iteration k0 + j.  At the end of a cycle the
// host solves the small triangular system R y = g and the device adds Z y to
// x; a restart begins from the true residual b - A_sigma x.
PcgOut gmres_run(ddeig_problem* P, int flags, const double* b, double* x, double rtol, int maxit,
                 int m) {
  const hipStream_t s = P->stream;
  const int batch = P->opt.batch_iters > 0 ? P->opt.batch_iters : 8;
  const GmWs w = gm_workspace(P, m);
  Red rr = slot(P, 1);
  launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
  launch_resid_init(P, b, P->q, P->r, rr, s);
  launch_pcg_init(P, rtol, rr, s);
  launch_gm_start(P, rr, P->r, w.V, w.g, w.gm, s);
  check_launch("gmres start");
  PcgState hs{};
  check_hip(hipMemcpyAsync(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s), "state");
  sync(P);
  int k = 0;
  std::vector<double> Hh, gh, yh;
  while (!hs.done && k < maxit) {
    const int kc0 = k;
    const int jmax = std::min(m, maxit - kc0);
    // steps j0..j1 on stream ms
    auto steps = [&](int j0, int j1, hipStream_t ms) {
      for (int j = j0; j <= j1; ++j) {
        const bool full = j < jmax;
        double* uj = w.V + (long)j * w.ldv;
        if (full) {
          double* zj = w.Z + (long)j * w.ldv;
          precond_apply(P, uj, zj, nullptr, P->st, nullptr, nullptr, nullptr, ms, flags);
          launch_stencil(P, P->tabAs, zj, w.w, nullptr, nullptr, ms);
        }
        launch_gm_dots(P, j, w.V, w.ldv, full ? w.w : nullptr, w.part, ms);
        launch_gm_sum(P, full ? 2 * j + 3 : j + 1, w.part, w.d, ms);
        launch_gm_decide(P, j, kc0 + j, maxit, m, full ? 1 : 0, w.d, w.H, w.cs, w.sn, w.g, w.cv,
                         w.gm, ms);
        if (full) launch_gm_update_basis(P, j, w.V, w.ldv, w.w, w.d, w.gm, ms);
      }
    };
    for (int j0 = 0; j0 <= jmax; j0 += batch) {
      const int j1 = std::min(jmax, j0 + batch - 1);
      if (P->opt.graphs) {
        // each block of steps is captured once per key and replayed on the library stream
        const auto key = std::make_tuple(kc0, j0, j1, jmax, maxit, m, flags, (const void*)w.V);
        auto it = P->gm_graphs.find(key);
        if (it == P->gm_graphs.end()) {
          if (P->gm_graphs.size() >= 4096) {
            for (auto& kv : P->gm_graphs) (void)hipGraphExecDestroy(kv.second);
            P->gm_graphs.clear();
          }
          it = P->gm_graphs
                   .emplace(key, capture_graph(P, [&](hipStream_t cs) { steps(j0, j1, cs); }))
                   .first;
        }
        check_hip(hipGraphLaunch(it->second, s), "launch graph");
      } else {
        steps(j0, j1, s);
      }
      check_launch("gmres step");
      check_hip(hipMemcpyAsync(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s), "state");
      sync(P);
      if (hs.done) break;
    }
    // columns completed in this cycle (a breakdown leaves its column out)
    const int jd = hs.iters - kc0 - (hs.done == 2 ? 1 : 0);
    k = hs.iters;
    if (jd > 0) {
      Hh.resize((size_t)(m + 1) * jd);
      gh.resize(jd);
      yh.resize(jd);
      check_hip(hipMemcpyAsync(Hh.data(), w.H, sizeof(double) * Hh.size(), hipMemcpyDeviceToHost,
                               s), "copy H");
      check_hip(hipMemcpyAsync(gh.data(), w.g, sizeof(double) * jd, hipMemcpyDeviceToHost, s),
                "copy g");
      sync(P);
      for (int i = jd - 1; i >= 0; --i) {  // R y = g, R upper triangular (column-major)
        double t = gh[i];
        for (int c = i + 1; c < jd; ++c) t -= Hh[(size_t)c * (m + 1) + i] * yh[c];
        yh[i] = t / Hh[(size_t)i * (m + 1) + i];
      }
      check_hip(hipMemcpyAsync(w.y, yh.data(), sizeof(double) * jd, hipMemcpyHostToDevice, s),
                "copy y");
      launch_gm_update(P, jd, w.Z, w.ldv, w.y, x, s);
      check_launch("gmres update");
      sync(P);
    }
    if (hs.done != 6) break;
    // restart from the true residual
    launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
    launch_resid_init(P, b, P->q, P->r, rr, s);
    launch_gm_start(P, rr, P->r, w.V, w.g, w.gm, s);
    check_launch("gmres restart");
    check_hip(hipMemcpyAsync(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost, s), "state");
    sync(P);
  }
  PcgOut o;
  o.iters = hs.iters;
  o.relres = hs.relres;
  o.done = hs.done == 6 ? 4 : (hs.done ? hs.done : 4);
  return o;
}

// Eigen-decomposition of a symmetric 3 x 3 matrix by cyclic Jacobi rotations
// (FP64, fixed sweep order); ev ascending, V's columns the eigenvectors.
void sym3_eig(const double Ain[3][3], double ev[3], double V[3][3]) {
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[i][j] = 0.5 * (Ain[i][j] + Ain[j][i]);
      V[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    const double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
    const double dia = std::fabs(A[0][0]) + std::fabs(A[1][1]) + std::fabs(A[2][2]);
    if (off <= 1e-18 * dia || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {  // A := A J on columns p, q
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A := J^T A on rows p, q
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  int ord[3] = {0, 1, 2};
  std::sort(ord, ord + 3, [&](int a, int b) { return A[a][a] < A[b][b]; });
  double W[3][3];
  for (int j = 0; j < 3; ++j) {
    ev[j] = A[ord[j]][ord[j]];
    for (int k = 0; k < 3; ++k) W[k][j] = V[k][ord[j]];
  }
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) V[k][j] = W[k][j];
}

// Rayleigh-Ritz in span(S) from its Gram matrices: GA[i][j] = s_i^T A s_j,
// GB[i][j] = s_i^T B s_j.  Columns are scaled to unit B-norm (zero columns
// ignored), directions with scaled Gram eigenvalue <= 1e-10 of the largest
// are dropped, and c receives the coefficients of the minimiser (not normalised).
void rayleigh_ritz3(const double GA[3][3], const double GB[3][3], double c[3]) {
  double sc[3];
  for (int i = 0; i < 3; ++i) sc[i] = GB[i][i] > 0.0 ? 1.0 / std::sqrt(GB[i][i]) : 0.0;
  double gb[3][3], ga[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gb[i][j] = GB[i][j] * sc[i] * sc[j];
      ga[i][j] = GA[i][j] * sc[i] * sc[j];
    }
  double ev[3], V[3][3];
  sym3_eig(gb, ev, V);
  double T[3][3];
  int nk = 0;
  for (int j = 0; j < 3; ++j)
    if (ev[j] > 1e-10 * ev[2]) {
      for (int k = 0; k < 3; ++k) T[k][nk] = V[k][j] / std::sqrt(ev[j]);
      ++nk;
    }
  double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < nk; ++a)
    for (int b = 0; b < nk; ++b) {
      double v = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v += T[i][a] * ga[i][j] * T[j][b];
      H[a][b] = v;
    }
  // unused directions get a large diagonal so that they are never the minimiser
  double big = 1.0;
  for (int a = 0; a < nk; ++a) big += std::fabs(H[a][a]);
  for (int a = nk; a < 3; ++a) H[a][a] = 1e3 * big;
  double mu[3], Y[3][3];
  sym3_eig(H, mu, Y);
  for (int i = 0; i < 3; ++i) {
    double v = 0.0;
    for (int a = 0; a < nk; ++a) v += T[i][a] * Y[a][0];
    c[i] = sc[i] * v;
  }
}

// Validated device description of a potential (see ddeig_potential).
ddeig_status make_vspec(const ddeig_potential* V, int p, int q, double ell, ddeig::VSpec& vs) {
  if (V->nterms < 0 || V->nterms > DDEIG_MAX_TERMS)
    return set_error(DDEIG_EINVAL, "nterms out of range");
  if ((int)V->kind < 0 || (int)V->kind > 5) return set_error(DDEIG_EINVAL, "unknown potential kind");
  if (V->kind == DDEIG_V_FOURIER2 && p != 2)
    return set_error(DDEIG_EINVAL, "FOURIER2 potentials need p = 2");
  vs.kind = (int)V->kind;
  vs.nterms = V->nterms;
  vs.p = p;
  vs.q = q;
  vs.cy = V->cy;
  vs.c0 = V->c0;
  vs.ell = ell;
  const bool needs_terms = V->kind == DDEIG_V_SEP_FOURIER || V->kind == DDEIG_V_FOURIER2 ||
                           V->kind == DDEIG_V_SEP_SUM;
  if (needs_terms && V->nterms > 0) {
    if (V->a == nullptr || V->k == nullptr) return set_error(DDEIG_EINVAL, "potential arrays are NULL");
    if ((V->kind != DDEIG_V_SEP_SUM) && V->phi == nullptr)
      return set_error(DDEIG_EINVAL, "potential phases are NULL");
    if ((V->kind == DDEIG_V_FOURIER2 || V->kind == DDEIG_V_SEP_SUM) && V->m == nullptr)
      return set_error(DDEIG_EINVAL, "potential m array is NULL");
    for (int t = 0; t < V->nterms; ++t) {
      vs.a[t] = V->a[t];
      vs.phi[t] = V->phi ? V->phi[t] : 0.0;
      vs.k[t] = V->k[t];
      vs.m[t] = V->m ? V->m[t] : 0;
      if (!std::isfinite(vs.a[t]) || !std::isfinite(vs.phi[t]))
        return set_error(DDEIG_EINVAL, "non-finite potential coefficient");
      if (V->kind == DDEIG_V_SEP_SUM && (vs.m[t] < 0 || vs.m[t] >= p + q))
        return set_error(DDEIG_EINVAL, "SEP_SUM axis out of range");
    }
  }
  if (V->kind == DDEIG_V_SEP_SUM && V->g != nullptr)
    for (int j = 0; j < q; ++j) vs.g[j] = V->g[j];
  if (!std::isfinite(vs.cy) || !std::isfinite(vs.c0)) return set_error(DDEIG_EINVAL, "non-finite cy/c0");
  vs.table = nullptr;  // QUAD_TABLE: the caller sets the device copy (quad_table_len, upload)
  return DDEIG_OK;
}

// Length of a QUAD_TABLE potential on the period cell of (p, q, n_e, ell).
long quad_table_len(int p, int q, int ne, double ell) {
  long len = 1L << (p + q);
  for (int a = 0; a < p; ++a) len *= ne;
  const long ely = std::lround(ell * ne);
  for (int a = 0; a < q; ++a) len *= ely;
  return len;
}

ddeig_status check_quad_table(const ddeig_potential* V, long expect) {
  if (V->kind != DDEIG_V_QUAD_TABLE) return DDEIG_OK;
  if (V->table == nullptr) return set_error(DDEIG_EINVAL, "QUAD_TABLE potential without a table");
  if (V->table_len != expect)
    return set_error(DDEIG_EINVAL, "QUAD_TABLE length is " + std::to_string(V->table_len) +
                                       ", the period cell has " + std::to_string(expect) +
                                       " quadrature points");
  for (long i = 0; i < expect; ++i)
    if (!std::isfinite(V->table[i])) return set_error(DDEIG_EINVAL, "non-finite QUAD_TABLE value");
  return DDEIG_OK;
}

ddeig_status validate_vec(const void* p, const char* name) {
  if (p == nullptr) return set_error(DDEIG_EINVAL, std::string(name) + " is NULL");
  return DDEIG_OK;
}

}  // namespace

namespace ddeig {
void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Failure{DDEIG_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
  }
}
}  // namespace ddeig

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                                  \
  }                                                                    \
  catch (const Failure& f) {                                           \
    return set_error(f.status, f.msg);                                 \
  }                                                                    \
  catch (const std::bad_alloc&) {                                      \
    return set_error(DDEIG_ENOMEM, "host allocation failed");          \
  }                                                                    \
  catch (...) {                                                        \
    return set_error(DDEIG_EINTERNAL, "unexpected internal exception"); \
  }

extern "C" {

const char* ddeig_status_string(ddeig_status s) {
  switch (s) {
    case DDEIG_OK: return "ok";
    case DDEIG_EINVAL: return "invalid argument";
    case DDEIG_ENOMEM: return "out of memory";
    case DDEIG_EHIP: return "HIP runtime error";
    case DDEIG_ENOTSPD: return "operator or preconditioner not positive definite";
    case DDEIG_ENOCONV: return "iteration limit reached";
    case DDEIG_ESTATE: return "call order violated";
    case DDEIG_EINTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* ddeig_last_error(void) { return g_last_error.c_str(); }

ddeig_status ddeig_assemble(const ddeig_geometry* geom, double h, const ddeig_potential* V,
                            int overlap, const ddeig_options* opts, void* hip_stream,
                            ddeig_problem** out) {
  if (out == nullptr) return set_error(DDEIG_EINVAL, "out is NULL");
  *out = nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  if (geom == nullptr || V == nullptr) return set_error(DDEIG_EINVAL, "geometry or potential is NULL");
  const int p = geom->p, q = geom->q, L = geom->L;
  if (p < 1 || q < 1 || p + q < 2 || p + q > 3)
    return set_error(DDEIG_EINVAL, "need p >= 1, q >= 1 and p + q in {2, 3}");
  if (L < 1) return set_error(DDEIG_EINVAL, "L must be >= 1");
  if (!std::isfinite(h) || h <= 0.0) return set_error(DDEIG_EINVAL, "h must be positive and finite");
  const double ne_d = 1.0 / h;
  const long ne_l = std::lround(ne_d);
  if (std::fabs(ne_d - (double)ne_l) > 1e-12 * ne_d || ne_l < 3 || ne_l > 4096)
    return set_error(DDEIG_EINVAL, "1/h must be an integer n_e with 3 <= n_e <= 4096");
  const int ne = (int)ne_l;
  const double ell = geom->ell;
  if (!std::isfinite(ell) || ell <= 0.0) return set_error(DDEIG_EINVAL, "ell must be positive");
  const double elne_d = ell * ne;
  const long elne = std::lround(elne_d);
  if (std::fabs(elne_d - (double)elne) > 1e-9 * elne_d || elne < 2)
    return set_error(DDEIG_EINVAL, "ell * n_e must be an integer >= 2");
  if (overlap < 1 || 2 * overlap > ne)
    return set_error(DDEIG_EINVAL, "overlap must satisfy 1 <= overlap and 2 overlap <= n_e");
  ddeig_options o{0, 1, 0, 8, 0, 0};
  if (opts) o = *opts;
  if (o.pu < 0 || o.pu > 1 || o.coarse < 0 || o.coarse > 1 || o.local_prec < 0 ||
      o.local_prec > 3 || o.batch_iters < 0 || o.graphs < 0 || o.graphs > 1 || o.sweep < 0 ||
      o.sweep > 2)
    return set_error(DDEIG_EINVAL, "invalid options");

  ddeig::VSpec vs{};
  {
    const ddeig_status sv = make_vspec(V, p, q, ell, vs);
    if (sv != DDEIG_OK) return sv;
    const ddeig_status st = check_quad_table(V, quad_table_len(p, q, ne, ell));
    if (st != DDEIG_OK) return st;
  }

  ddeig::Geo g{};
  g.p = p; g.q = q; g.D = p + q; g.L = L; g.ne = ne;
  g.h = 1.0 / ne; g.ell = ell;
  g.ntaps = g.D == 2 ? 9 : 27;
  long n = 1, ts = 1;
  for (int a = 0; a < 3; ++a) {
    if (a >= g.D) {
      g.nel[a] = 1; g.N[a] = 1; g.P[a] = 1; g.isx[a] = 0;
      continue;
    }
    g.isx[a] = a < p;
    g.nel[a] = g.isx[a] ? L * ne : (int)elne;
    g.N[a] = g.nel[a] - 1;
    g.P[a] = g.isx[a] ? ne : g.N[a];
    n *= g.N[a];
    ts *= g.P[a];
  }
  if (n < 1) return set_error(DDEIG_EINVAL, "no interior unknowns");
  if (n > (1L << 34)) return set_error(DDEIG_EINVAL, "problem too large");
  g.n = n;
  g.tsize = ts;
  g.fN0 = ddeig::make_fastdiv((unsigned)g.N[0]);
  g.fN1 = ddeig::make_fastdiv((unsigned)g.N[1]);
  g.fne = ddeig::make_fastdiv((unsigned)ne);

  ddeig_problem* P = new (std::nothrow) ddeig_problem();
  if (!P) return set_error(DDEIG_ENOMEM, "host allocation failed");
  P->g = g;
  P->vs = vs;
  P->delta = overlap;
  P->opt = o;
  P->stream = static_cast<hipStream_t>(hip_stream);
  try {
    check_hip(hipGetDevice(&P->device), "hipGetDevice");
    // the scratch of the no-allocation entry point on this device (looked up
    // once per device; a failure is reported by that entry point)
    (void)ddeig::noalloc_init(P->device);
    const hipStream_t s = P->stream;
    const long tt = g.tsize * g.ntaps;
    P->tabK = dalloc<double>(P, tt);
    P->tabM = dalloc<double>(P, tt);
    P->tabA = dalloc<double>(P, tt);
    P->tabAs = dalloc<double>(P, tt);
    P->dVS = dalloc<ddeig::VSpec>(P, 1);
    P->dWS = dalloc<ddeig::VSpec>(P, 1);
    if (V->kind == DDEIG_V_QUAD_TABLE) {
      P->vtab_host.assign(V->table, V->table + V->table_len);
      P->dVtab = dalloc<double>(P, (size_t)V->table_len);
      check_hip(hipMemcpy(P->dVtab, V->table, sizeof(double) * V->table_len,
                          hipMemcpyHostToDevice), "copy potential table");
      P->vs.table = P->dVtab;
    }
    P->tabW = dalloc<double>(P, tt);
    check_hip(hipMemcpyAsync(P->dVS, &P->vs, sizeof(ddeig::VSpec), hipMemcpyHostToDevice, s), "copy V");
    launch_build_tables(P, s);
    check_launch("build tables");

    // decomposition into the L^p unit cells with `overlap` layers (§3, §4.1)
    const int nsub = p == 1 ? L : L * L;
    P->nsub = nsub;
    std::map<std::vector<int>, int> type_of;
    P->subs.resize(nsub);
    for (int sid = 0; sid < nsub; ++sid) {
      int c[3] = {sid % L + 1, p == 2 ? sid / L + 1 : 0, 0};
      ddeig::SubDev sd{};
      Box bx{};
      std::vector<int> key;
      for (int a = 0; a < 3; ++a) {
        bx.per[a] = 0;
        if (a >= g.D) { bx.o[a] = 0; bx.m[a] = 1; continue; }
        if (g.isx[a]) {
          const int lo = std::max((c[a] - 1) * ne - overlap + 1, 1);
          const int hi = std::min(c[a] * ne + overlap - 1, L * ne - 1);
          bx.o[a] = lo - 1;
          bx.m[a] = hi - lo + 1;
          const int cls = (L == 1) ? 3 : (c[a] == 1 ? 0 : (c[a] == L ? 2 : 1));
          key.push_back(cls);
        } else {
          bx.o[a] = 0;
          bx.m[a] = g.N[a];
        }
      }
      bx.b = 1;
      for (int a = 0; a < g.D - 1; ++a) bx.b *= bx.m[a];
      bx.nch = bx.m[g.D - 1];
      for (int a = 0; a < 3; ++a) { sd.o[a] = bx.o[a]; sd.c[a] = c[a]; }
      auto it = type_of.find(key);
      int tid;
      if (it == type_of.end()) {
        tid = (int)P->types.size();
        type_of[key] = tid;
        ddeig::SubType t;
        t.box = bx;
        t.nmem = 0;
        P->types.push_back(t);
      } else {
        tid = it->second;
      }
      auto& T = P->types[tid];
      sd.type = tid;
      sd.slot = T.nmem++;
      T.members.push_back(sid);
      P->subs[sid] = sd;
    }
    int maxb = 0;
    std::vector<ddeig::TypeDev> tdev(P->types.size());
    const bool dense = o.local_prec >= 2;
    std::vector<ddeig::GemmTile> tiles;
    std::vector<ddeig::GemvRows> gemv;
    std::vector<ddeig::EmbedJob> embjobs;
    if (dense) {
      // the unclipped box of an interior cell (o = n_e - delta in x dims, the
      // box of cell 2; only the table is read, so it exists for any L)
      ddeig::DenseHost& H = P->dh;
      Box hb{};
      for (int a = 0; a < 3; ++a) {
        hb.per[a] = 0;
        if (a >= g.D) { hb.o[a] = 0; hb.m[a] = 1; continue; }
        if (g.isx[a]) { hb.o[a] = ne - overlap; hb.m[a] = ne + 2 * overlap - 1; }
        else { hb.o[a] = 0; hb.m[a] = g.N[a]; }
      }
      hb.b = 1;
      for (int a = 0; a < g.D - 1; ++a) hb.b *= hb.m[a];
      hb.nch = hb.m[g.D - 1];
      H.box = hb;
      H.m = hb.b * hb.nch;
      H.ld = (H.m + 127) / 128 * 128;
      H.mp = nsub > ddeig::kGemvMax ? (nsub + 127) / 128 * 128 : ddeig::kGemvMax;
      H.W = dalloc<double>(P, (size_t)hb.nch * hb.b * hb.b);
      const size_t aa = (size_t)H.ld * H.ld, rr = (size_t)H.mp * H.ld;
      // K columns per GEMM stage (the kernel's pipeline depth): 64 with a
      // single bf16 inverse, 32 with the hi/lo pair; K split so that the GEMM
      // has about one workgroup per CU, at even stage counts (the kernel
      // multiplies two stages per trip)
      const int bk = o.local_prec == 2 ? 32 : 64;
      if (nsub > ddeig::kGemvMax) {
        const long ntile = (long)(H.mp / 128) * (H.ld / 128);
        P->ksplit = (int)std::max<long>(1, std::min<long>(std::min(3, H.ld / bk / 2),
                                                          (256 + ntile - 1) / ntile));
      } else {
        P->ksplit = 1;
      }
      H.Ah = dalloc<__bf16>(P, aa);
      H.Al = o.local_prec == 2 ? dalloc<__bf16>(P, aa) : nullptr;
      H.Rh = dalloc<__bf16>(P, rr);
      H.Rl = o.local_prec == 2 ? dalloc<__bf16>(P, rr) : nullptr;
      H.Z = dalloc<float>(P, (size_t)P->ksplit * rr);
      // rows are zero outside each member's own box, and padding rows stay zero
      check_hip(hipMemsetAsync(H.Rh, 0, rr * sizeof(__bf16), s), "memset Rh");
      if (H.Rl) check_hip(hipMemsetAsync(H.Rl, 0, rr * sizeof(__bf16), s), "memset Rl");
      maxb = std::max(maxb, hb.b);
      // classes: their box inside the unclipped one, their rows, and for the
      // clipped ones the node list T of the unclipped box outside their box
      for (size_t t = 0; t < P->types.size(); ++t) {
        auto& T = P->types[t];
        const auto& sd0 = P->subs[T.members[0]];
        int nS = 1;
        for (int a = 0; a < 3; ++a) {
          T.off[a] = (a < g.D && g.isx[a]) ? T.box.o[a] - ((sd0.c[a] - 1) * ne - overlap) : 0;
          nS *= T.box.m[a];
          if (T.off[a] < 0 || T.off[a] + T.box.m[a] > hb.m[a])
            throw Failure{DDEIG_EINTERNAL, "subdomain box outside the unclipped box"};
        }
        const int nT = H.m - nS;
        if (nT > 0) {
          if (nT > ddeig::kEmbMaxT)
            throw Failure{DDEIG_EINVAL, "dense local solves: a clipped subdomain misses more than 1024 "
                                        "nodes of the unclipped box; use local_prec 0 or 1"};
          if ((long)nT * H.m >= (1L << 31))
            throw Failure{DDEIG_EINVAL, "dense local solves: a clipped-class correction matrix "
                                        "has 2^31 entries or more; use local_prec 0 or 1"};
          std::vector<int> tl;
          for (int u2 = 0; u2 < hb.m[2]; ++u2)
            for (int u1 = 0; u1 < hb.m[1]; ++u1)
              for (int u0 = 0; u0 < hb.m[0]; ++u0) {
                const int u[3] = {u0, u1, u2};
                bool in = true;
                for (int a = 0; a < 3; ++a)
                  if (u[a] < T.off[a] || u[a] >= T.off[a] + T.box.m[a]) in = false;
                if (!in) tl.push_back(u0 + hb.m[0] * (u1 + hb.m[1] * u2));
              }
          ddeig::EmbedDev E{};
          E.nT = nT;
          E.nmem = T.nmem;
          int* dR = dalloc<int>(P, T.members.size());
          check_hip(hipMemcpyAsync(dR, T.members.data(), sizeof(int) * T.members.size(),
                                   hipMemcpyHostToDevice, s), "copy member rows");
          E.rows = dR;
          for (int a = 0; a < 3; ++a) { E.off[a] = T.off[a]; E.m[a] = T.box.m[a]; }
          int* dT = dalloc<int>(P, tl.size());
          check_hip(hipMemcpyAsync(dT, tl.data(), sizeof(int) * tl.size(), hipMemcpyHostToDevice, s),
                    "copy T list");
          sync(P);  // tl is released at the end of this scope
          E.Tidx = dT;
          E.G = dalloc<float>(P, (size_t)nT * H.m);
          E.Z = H.Z;
          E.zsplit = (long)H.mp * H.ld;
          E.st = nullptr;
          E.xonly = (T.off[1] == 0 && T.box.m[1] == hb.m[1] && T.off[2] == 0 &&
                     T.box.m[2] == hb.m[2]) ? 1 : 0;
          if (E.xonly) {
            // the arithmetic T index must reproduce the list
            const int nmiss = hb.m[0] - T.box.m[0];
            for (int t = 0; t < nT; ++t) {
              const int line = t / nmiss, j = t - line * nmiss;
              const int u0 = j < T.off[0] ? j : j + T.box.m[0];
              if (u0 + hb.m[0] * line != tl[t]) {
                E.xonly = 0;
                break;
              }
            }
          }
          const int ci = (int)P->emb.size();
          P->emb.push_back(E);
          P->maxT = std::max(P->maxT, nT);
          const int per = ddeig::emb_members_per_job(nT);
          for (int m0 = 0; m0 < T.nmem; m0 += per)
            embjobs.push_back(ddeig::EmbedJob{ci, m0, std::min(per, T.nmem - m0)});
        }
      }
      // GEMM over all rows (or the streaming kernel for a handful of rows);
      // the tiles of one group read the same rows of the inverse
      if (nsub > ddeig::kGemvMax) {
        std::vector<std::vector<ddeig::GemmTile>> groups;
        const int npair = H.ld / bk / 2;
        for (int sp = 0; sp < P->ksplit; ++sp) {
          const int kb0 = 2 * (int)((long)npair * sp / P->ksplit);
          const int kb1 = 2 * (int)((long)npair * (sp + 1) / P->ksplit);
          for (int nt = 0; nt < H.ld / 128; ++nt) {
            std::vector<ddeig::GemmTile> grp;
            for (int mt = 0; mt < H.mp / 128; ++mt)
              grp.push_back(ddeig::GemmTile{0, mt * 128, nt * 128, kb0 * bk, kb1 * bk, sp});
            groups.push_back(grp);
          }
        }
        // workgroup i runs on XCD i mod 8: eight groups of equal size at a
        // time are interleaved so that the tiles of one group get ids 8 apart
        // and share that XCD's L2 copy of the inverse rows they read
        size_t gi = 0;
        while (gi < groups.size()) {
          size_t gj = gi;
          while (gj < groups.size() && gj - gi < 8 && groups[gj].size() == groups[gi].size()) ++gj;
          if (gj - gi == 8) {
            for (size_t i = 0; i < groups[gi].size(); ++i)
              for (size_t j = gi; j < gj; ++j) tiles.push_back(groups[j][i]);
          } else {
            for (size_t j = gi; j < gj; ++j)
              for (auto& tl : groups[j]) tiles.push_back(tl);
          }
          gi = gj;
        }
      } else {
        for (int r0 = 0; r0 < H.m; r0 += kBlock / 64)
          gemv.push_back(ddeig::GemvRows{0, r0, std::min(H.m, r0 + kBlock / 64), nsub});
      }
    }
    // FP64 / FP32 local solves of 3-D boxes: chain solves batched over the
    // members of a class (two launches per sweep step)
    int maxb_types = 0;
    for (auto& T : P->types) maxb_types = std::max(maxb_types, T.box.b);
    const bool batched_chain = !dense && g.D == 3;
    // FP32 factors of 3-D boxes: the chain solves run on MFMA
    bool chain_mfma = batched_chain && o.local_prec == 1;
    for (auto& T : P->types)
      if (!ddeig::chain_mfma_ok(T.box.b, T.box.m[0])) chain_mfma = false;
    P->chain_mfma = chain_mfma ? 1 : 0;
    std::vector<ddeig::ChainJob> chainjobs;
    int mtot = 0;
    for (size_t t = 0; t < P->types.size(); ++t) {
      auto& T = P->types[t];
      maxb = std::max(maxb, T.box.b);
      const long mm = (long)T.box.nch * T.box.b;
      const int ldw = chain_mfma ? (T.box.b + 3) / 4 * 4 : T.box.b;
      tdev[t].ldw = ldw;
      if (batched_chain) {
        const int mg = chain_mfma ? ddeig::chain_mfma_members() : ddeig::chain_group_members();
        for (int m0 = 0; m0 < T.nmem; m0 += mg)
          chainjobs.push_back(ddeig::ChainJob{(int)t, m0, std::min(mg, T.nmem - m0), mtot + m0});
        mtot += T.nmem;
      }
      for (int a = 0; a < 3; ++a) tdev[t].m[a] = T.box.m[a];
      tdev[t].b = T.box.b;
      tdev[t].nch = T.box.nch;
      for (int a = 0; a < 3; ++a) tdev[t].o[a] = T.box.o[a];
      tdev[t].tbatch = nullptr;
      tdev[t].dense = dense ? 1 : 0;
      if (dense) {
        const ddeig::DenseHost& H = P->dh;
        for (int a = 0; a < 3; ++a) {
          tdev[t].hm[a] = H.box.m[a];
          tdev[t].off[a] = T.off[a];
        }
        T.batch = dalloc<double>(P, 1);
        tdev[t].W = nullptr;
        tdev[t].W32 = nullptr;
        tdev[t].ld = H.ld;
        tdev[t].ksplit = P->ksplit;
        tdev[t].Rh = H.Rh;
        tdev[t].Rl = H.Rl;
        tdev[t].Z = H.Z;
        tdev[t].zsplit = (long)H.mp * H.ld;
      } else {
        T.W = dalloc<double>(P, (size_t)T.box.nch * T.box.b * T.box.b);
        if (o.local_prec == 1) T.W32 = dalloc<float>(P, (size_t)T.box.nch * T.box.b * ldw);
        T.batch = dalloc<double>(P, (size_t)T.nmem * mm);
        for (int a = 0; a < 3; ++a) {
          tdev[t].hm[a] = T.box.m[a];
          tdev[t].off[a] = 0;
        }
        if (batched_chain) tdev[t].tbatch = dalloc<double>(P, (size_t)T.nmem * mm);
        tdev[t].W = T.W;
        tdev[t].W32 = T.W32;
        tdev[t].ld = 0;
        tdev[t].ksplit = 0;
        tdev[t].Rh = tdev[t].Rl = nullptr;
        tdev[t].Z = nullptr;
        tdev[t].zsplit = 0;
      }
      tdev[t].batch = T.batch;
      T.phi = dalloc<double>(P, mm);
      tdev[t].phi = T.phi;
      tdev[t].fm0 = ddeig::make_fastdiv((unsigned)T.box.m[0]);
    }
    if (P->types.size() > (size_t)ddeig::kMaxTypes) throw Failure{DDEIG_EINTERNAL, "too many classes"};
    if (batched_chain) {
      P->chain_bmax = maxb_types;
      P->chain_mtot = mtot;
      P->chain_part = dalloc<unsigned char>(
          P, chain_mfma ? ddeig::chain_mfma_part_bytes(maxb_types, mtot)
                        : ddeig::chain_part_bytes(maxb_types, mtot, o.local_prec == 1));
      P->nchainjobs = (int)chainjobs.size();
      P->dChainJobs = dalloc<ddeig::ChainJob>(P, chainjobs.size());
      check_hip(hipMemcpyAsync(P->dChainJobs, chainjobs.data(),
                               sizeof(ddeig::ChainJob) * chainjobs.size(), hipMemcpyHostToDevice, s),
                "copy chain jobs");
      sync(P);  // chainjobs is released at the end of this scope
    }
    {
      std::vector<ddeig::SubTS> ts(nsub);
      for (int sid = 0; sid < nsub; ++sid) {
        const auto& sd = P->subs[sid];
        ts[sid] = ddeig::SubTS{sd.type, dense ? sid : sd.slot};
      }
      std::vector<int> first(P->types.size());
      std::vector<double*> phis(P->types.size());
      for (size_t t = 0; t < P->types.size(); ++t) {
        first[t] = P->types[t].members[0];
        phis[t] = P->types[t].phi;
      }
      P->dSubTS = dalloc<ddeig::SubTS>(P, nsub);
      P->dFirst = dalloc<int>(P, first.size());
      P->dPhis = dalloc<double*>(P, phis.size());
      check_hip(hipMemcpyAsync(P->dSubTS, ts.data(), sizeof(ddeig::SubTS) * nsub,
                               hipMemcpyHostToDevice, s), "copy sub table");
      check_hip(hipMemcpyAsync(P->dFirst, first.data(), sizeof(int) * first.size(),
                               hipMemcpyHostToDevice, s), "copy first members");
      check_hip(hipMemcpyAsync(P->dPhis, phis.data(), sizeof(double*) * phis.size(),
                               hipMemcpyHostToDevice, s), "copy phi pointers");
      sync(P);
    }
    if (dense) {
      const ddeig::DenseHost& H = P->dh;
      P->ntiles = (int)tiles.size();
      P->ngemv = (int)gemv.size();
      P->dGemv = dalloc<ddeig::GemvRows>(P, std::max<size_t>(gemv.size(), 1));
      if (!gemv.empty())
        check_hip(hipMemcpyAsync(P->dGemv, gemv.data(), sizeof(ddeig::GemvRows) * gemv.size(),
                                 hipMemcpyHostToDevice, s), "copy gemv rows");
      P->dTiles = dalloc<ddeig::GemmTile>(P, std::max<size_t>(tiles.size(), 1));
      if (!tiles.empty())
        check_hip(hipMemcpyAsync(P->dTiles, tiles.data(), sizeof(ddeig::GemmTile) * tiles.size(),
                                 hipMemcpyHostToDevice, s), "copy tiles");
      const ddeig::GemmType gt{H.Ah, H.Al, H.Rh, H.Rl, H.Z, (long)H.mp * H.ld, H.ld, nsub, nullptr};
      P->dGtypes = dalloc<ddeig::GemmType>(P, 1);
      check_hip(hipMemcpyAsync(P->dGtypes, &gt, sizeof(ddeig::GemmType), hipMemcpyHostToDevice, s),
                "copy gemm operands");
      if (embjobs.size() > (size_t)ddeig::kEmbMaxJobs)
        throw Failure{DDEIG_EINVAL, "dense local solves: more than 65535 clipped-subdomain "
                                    "correction jobs; use local_prec 0 or 1"};
      P->nembjobs = (int)embjobs.size();
      if (!P->emb.empty()) {
        P->dEmb = dalloc<ddeig::EmbedDev>(P, P->emb.size());
        check_hip(hipMemcpyAsync(P->dEmb, P->emb.data(), sizeof(ddeig::EmbedDev) * P->emb.size(),
                                 hipMemcpyHostToDevice, s), "copy clipped classes");
        P->dEmbJobs = dalloc<ddeig::EmbedJob>(P, embjobs.size());
        check_hip(hipMemcpyAsync(P->dEmbJobs, embjobs.data(),
                                 sizeof(ddeig::EmbedJob) * embjobs.size(), hipMemcpyHostToDevice, s),
                  "copy correction jobs");
      }
      sync(P);  // the host vectors above are released at the end of this scope
    }
    P->maxb = std::max(maxb, 1);
    const Box cb = cell_box(g);
    const int gjmax = std::max(std::max(std::max(maxb, cb.b), nsub), P->maxT);
    P->dSubs = dalloc<ddeig::SubDev>(P, nsub);
    P->dTypes = dalloc<ddeig::TypeDev>(P, tdev.size());
    check_hip(hipMemcpyAsync(P->dSubs, P->subs.data(), sizeof(ddeig::SubDev) * nsub,
                             hipMemcpyHostToDevice, s), "copy subdomains");
    check_hip(hipMemcpyAsync(P->dTypes, tdev.data(), sizeof(ddeig::TypeDev) * tdev.size(),
                             hipMemcpyHostToDevice, s), "copy types");
    P->r = dalloc<double>(P, n);
    P->z = dalloc<double>(P, n);
    P->pp[0] = dalloc<double>(P, n);
    P->pp[1] = dalloc<double>(P, n);
    P->q = dalloc<double>(P, n);
    P->u = dalloc<double>(P, n);
    P->tmpv = dalloc<double>(P, std::max<long>(n, g.tsize));
    P->w = dalloc<double>(P, n);
    P->red_part = dalloc<double>(P, (size_t)kRedSlots * kMaxRed);
    P->big_cap = ddeig::stencil_tiles(g);
    if (P->big_cap > kMaxRed) P->big_part = dalloc<double>(P, 2 * (size_t)P->big_cap);
    P->red_val = dalloc<double>(P, kRedSlots);
    P->st = dalloc<ddeig::PcgState>(P, 1);
    P->hist_cap = 10001;
    P->hist = dalloc<double>(P, P->hist_cap);
    P->scal = dalloc<double>(P, 8);
    P->flag = dalloc<int>(P, 1);
    check_hip(hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking), "create stream");
    if (o.graphs)
      check_hip(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking), "create capture stream");
    check_hip(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming), "create event");
    check_hip(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming), "create event");
    for (int e = 0; e < 2; ++e)
      check_hip(hipEventCreateWithFlags(&P->ev_state[e], hipEventDisableTiming), "create event");
    check_hip(hipHostMalloc(reinterpret_cast<void**>(&P->hst), 2 * sizeof(ddeig::PcgState)),
              "pinned state");
    P->gjbuf = dalloc<double>(P, 4 * (size_t)gjmax);
    P->gj_stride = gjmax;
    P->psi = dalloc<double>(P, g.tsize);
    P->crhs = dalloc<double>(P, nsub);
    // per-axis covering tables of the expanding directions
    for (int a = 0; a < p; ++a) {
      std::vector<ddeig::XCover> xc(g.N[a]);
      for (int i = 0; i < g.N[a]; ++i) {
        const int gi = i + 1;
        const int num = gi - overlap + 1;
        int clo = num <= 0 ? 1 : (num + ne - 1) / ne;
        int chi = (gi + overlap - 1) / ne + 1;
        clo = std::max(clo, 1);
        chi = std::min(chi, L);
        ddeig::XCover c{};
        long dsum = 0;
        long dist[2] = {0, 0};
        for (int q2 = 0; q2 < 2; ++q2) {
          const int cc = clo + q2;
          if (cc > chi) { c.c[q2] = 0; c.u[q2] = 0; c.w[q2] = 0.0; continue; }
          c.c[q2] = cc;
          const int lo = std::max((cc - 1) * ne - overlap + 1, 1);
          c.u[q2] = i - (lo - 1);
          long dm = -1;  // distance (in units of h) to the interior faces of the box
          if (cc > 1) dm = gi - ((cc - 1) * ne - overlap);
          if (cc < L) {
            const long dh = (long)cc * ne + overlap - gi;
            dm = dm < 0 ? dh : std::min(dm, dh);
          }
          dist[q2] = dm;
          dsum += dm;
        }
        const int cnt = chi - clo + 1;
        for (int q2 = 0; q2 < cnt; ++q2) {
          if (o.pu == 0 || L == 1) c.w[q2] = 1.0 / cnt;
          else c.w[q2] = (double)dist[q2] / (double)dsum;
        }
        xc[i] = c;
      }
      P->dXC[a] = dalloc<ddeig::XCover>(P, xc.size());
      check_hip(hipMemcpyAsync(P->dXC[a], xc.data(), sizeof(ddeig::XCover) * xc.size(),
                               hipMemcpyHostToDevice, s), "copy covering table");
      sync(P);  // xc is released at the end of this scope
    }
    if (p == 1) P->dXC[1] = P->dXC[0];  // unused second axis
    P->cy = dalloc<double>(P, nsub);
    P->cfield = dalloc<double>(P, p == 1 ? (size_t)g.N[0] : (size_t)g.N[0] * g.N[1]);
    P->A0inv = dalloc<double>(P, (size_t)nsub * nsub);
    check_hip(hipMemsetAsync(P->flag, 0, sizeof(int), s), "memset flag");
    check_hip(hipMemsetAsync(P->psi, 0, sizeof(double) * g.tsize, s), "memset psi");
    sync(P);
  } catch (const Failure& f) {
    ddeig_destroy(P);
    return set_error(f.status, f.msg);
  } catch (...) {
    ddeig_destroy(P);
    return set_error(DDEIG_EINTERNAL, "unexpected exception in assemble");
  }
  P->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                            t_start).count();
  *out = P;
  return DDEIG_OK;
}

void ddeig_destroy(ddeig_problem* P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  clear_graphs(P);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  if (P->aux) {
    (void)hipStreamSynchronize(P->aux);
    (void)hipStreamDestroy(P->aux);
  }

  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  for (int e = 0; e < 2; ++e)
    if (P->ev_state[e]) (void)hipEventDestroy(P->ev_state[e]);
  if (P->hst) (void)hipHostFree(P->hst);
  for (void* p : P->allocs) (void)hipFree(p);
  P->allocs.clear();
  delete P;
}

ddeig_status ddeig_lopcg(ddeig_problem* P, double* x, const double* x_prev, double tol_o,
                         int maxit_outer, int mode, int inner, double rtol_inner, int maxit_inner,
                         ddeig_lopcg_info* info) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(x, "x")) return DDEIG_EINVAL;
  if (x_prev != nullptr && x_prev == x) return set_error(DDEIG_EINVAL, "x and x_prev must not alias");
  if (!(tol_o >= 0.0) || !std::isfinite(tol_o) || maxit_outer < 1 || mode < 0 || mode > 2 ||
      (mode == 0 && (!(rtol_inner >= 0.0) || !std::isfinite(rtol_inner))) ||
      (mode < 2 && maxit_inner < 1))
    return set_error(DDEIG_EINVAL, "invalid tolerances, iteration limits or mode");
  if (inner < DDEIG_INNER_CG_AS2 || inner > DDEIG_INNER_RAS1 ||
      (mode == 2 && inner > DDEIG_INNER_GMRES_RAS2))
    return set_error(DDEIG_EINVAL, "invalid inner solver for this mode");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "lopcg before the shift is set");
  if ((inner == DDEIG_INNER_GMRES_RAS2 || inner == DDEIG_INNER_RAS2) && !P->opt.coarse)
    return set_error(DDEIG_ESTATE, "the problem was assembled without the coarse space");
  API_GUARD_BEGIN
  const hipStream_t s = P->stream;
  const long n = P->g.n;
  const auto t0 = std::chrono::steady_clock::now();
  if (!P->lv) {
    P->lv = dalloc<double>(P, 9 * (size_t)n);
    P->lvp = dalloc<double*>(P, 9);
    P->lpart = dalloc<double>(P, (size_t)kLopcgQ * kMaxRed);
    P->lout = dalloc<double>(P, 16);
  }
  double* W = P->lv;
  double* AX = P->lv + n;
  double* BX = P->lv + 2 * n;
  double* XP = P->lv + 3 * n;
  double* AXP = P->lv + 4 * n;
  double* BXP = P->lv + 5 * n;
  double* AW = P->lv + 6 * n;
  double* BW = P->lv + 7 * n;
  double* R = P->lv + 8 * n;
  // pointer table {x, w, p, Ax, Aw, Ap, Bx, Bw, Bp} (p lives in the x_{k-1} buffers)
  double* tab[9] = {x, W, XP, AX, AW, AXP, BX, BW, BXP};
  check_hip(hipMemcpyAsync(P->lvp, tab, sizeof(tab), hipMemcpyHostToDevice, s), "copy pointers");
  auto read = [&](int cnt, double* h) {
    check_hip(hipMemcpyAsync(h, P->lout, sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "copy");
    sync(P);
  };
  // x_1 (constant if zero) and x_0 (first unit vector if not given), M-normalised
  Red s3 = slot(P, 3);
  launch_dot(x, x, n, s3, s);
  if (host_sum(P, s3) == 0.0) launch_fill(x, n, 1.0, s);
  if (x_prev) {
    launch_copy(XP, x_prev, n, s);
  } else {
    launch_fill(XP, n, 0.0, s);
    const double one = 1.0;
    check_hip(hipMemcpyAsync(XP, &one, sizeof(double), hipMemcpyHostToDevice, s), "unit vector");
    sync(P);
  }
  for (double* v : {x, XP}) {
    launch_stencil(P, P->tabM, v, W, &s3, nullptr, s);  // partials of v^T M v
    launch_scale_copy(n, v, v, s3, s);
  }
  Red s4 = slot(P, 4);
  launch_stencil(P, P->tabA, x, AX, &s4, nullptr, s);  // x^T A x
  launch_stencil(P, P->tabM, x, BX, nullptr, nullptr, s);
  double lam = host_sum(P, s4);
  double h[kLopcgQ];
  launch_lopcg_resid(n, lam, AX, BX, R, P->lpart, P->lout, s);
  read(1, h);
  double res = std::sqrt(std::max(h[0], 0.0));
  long inner_sum = 0;
  int inner_max = 0, k = 1;
  ddeig_status st = DDEIG_OK;
  while (res > tol_o && k <= maxit_outer) {
    // inner step: w ~ A_sigma^{-1} r
    launch_fill(W, n, 0.0, s);
    int its = 1;
    if (mode == 2) {
      precond_apply(P, R, W, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                    inner == DDEIG_INNER_GMRES_RAS2 ? kPrecLocal | kPrecCoarse | kPrecRas : -1);
    } else {
      // the inner solve; reaching maxit_inner is not an error (the outer
      // iteration goes on with the last inner iterate, as in §4.2)
      const double rt = mode == 0 ? rtol_inner : std::min(0.1, res);
      PcgOut o;
      if (inner == DDEIG_INNER_CG_AS2)
        o = pcg_run(P, R, W, rt, maxit_inner);
      else if (inner == DDEIG_INNER_GMRES_RAS2)
        o = gmres_run(P, kPrecLocal | kPrecCoarse | kPrecRas, R, W, rt, maxit_inner,
                      std::min(maxit_inner, 300));
      else
        o = sras_run(P, inner == DDEIG_INNER_RAS2 ? 2 : 1, R, W, rt, maxit_inner);
      if (inner == DDEIG_INNER_CG_AS2 && (o.done == 2 || o.done == 3)) {
        st = set_error(DDEIG_ENOTSPD, "CG breakdown inside LOPCG");
        break;
      }
      if (o.done == 2) {
        st = set_error(DDEIG_ENOCONV, inner == DDEIG_INNER_GMRES_RAS2
                                          ? "GMRES breakdown inside LOPCG"
                                          : "the stationary RAS inner solve diverged");
        break;
      }
      its = o.iters;
    }
    inner_sum += its;
    inner_max = std::max(inner_max, its);
    // B-orthogonalise w and p = x_k - x_{k-1} against x_k on the vectors,
    // then their A and B images, then the Gram data
    Red s5 = slot(P, 5), s6 = slot(P, 6);
    launch_dot(BX, W, n, s5, s);
    launch_dot(BX, XP, n, s6, s);
    const double alpha = host_sum(P, s5), beta = host_sum(P, s6);
    launch_lopcg_orth(n, alpha, beta, x, W, XP, s);
    launch_stencil(P, P->tabA, W, AW, nullptr, nullptr, s);
    launch_stencil(P, P->tabM, W, BW, nullptr, nullptr, s);
    launch_stencil(P, P->tabA, XP, AXP, nullptr, nullptr, s);
    launch_stencil(P, P->tabM, XP, BXP, nullptr, nullptr, s);
    launch_lopcg_gram(n, P->lvp, P->lpart, P->lout, s);
    read(kLopcgQ, h);
    const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    double GA[3][3], GB[3][3];
    for (int q = 0; q < 6; ++q) {
      const int a = ij[q][0], b = ij[q][1];
      GA[a][b] = GA[b][a] = h[q];
      GB[a][b] = GB[b][a] = h[6 + q];
    }
    double c[3];
    rayleigh_ritz3(GA, GB, c);
    double nrm = 0.0, sgn = 0.0;
    for (int a = 0; a < 3; ++a) {
      sgn += c[a] * h[12 + a];
      for (int b = 0; b < 3; ++b) nrm += c[a] * GB[a][b] * c[b];
    }
    if (!(nrm > 0.0)) {
      st = set_error(DDEIG_ENOTSPD, "LOPCG: the Ritz vector has no positive M-norm");
      break;
    }
    const double f = (sgn < 0.0 ? -1.0 : 1.0) / std::sqrt(nrm);
    launch_lopcg_update(n, f * c[0], f * c[1], f * c[2], x, W, XP, s);
    Red s7 = slot(P, 7);
    launch_stencil(P, P->tabA, x, AX, &s7, nullptr, s);  // x^T A x
    launch_stencil(P, P->tabM, x, BX, nullptr, nullptr, s);
    lam = host_sum(P, s7);
    launch_lopcg_resid(n, lam, AX, BX, R, P->lpart, P->lout, s);
    read(1, h);
    res = std::sqrt(std::max(h[0], 0.0));
    ++k;
  }
  check_launch("lopcg");
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->lambda = lam;
    info->res_norm = res;
    info->outer_its = k - 1;
    info->inner_sum = inner_sum;
    info->inner_max = inner_max;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  if (st != DDEIG_OK) return st;
  if (res > tol_o) return set_error(DDEIG_ENOCONV, "LOPCG reached maxit_outer");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_profile_kernel(ddeig_problem* P, int which, int reps, const double* x, double* y,
                                  double* avg_us, double* work) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (reps < 1 || which < 0 || which > 5 || !avg_us) return set_error(DDEIG_EINVAL, "invalid arguments");
  if (which != 1 && which != 5 && (validate_vec(x, "x") || validate_vec(y, "y"))) return DDEIG_EINVAL;
  if (!P->shifted) return set_error(DDEIG_ESTATE, "profile_kernel before the shift is set");
  API_GUARD_BEGIN
  const hipStream_t s = P->stream;
  double w = 0.0;
  if (which == 0) {
    w = 16.0 * (double)P->g.n;
  } else if (which == 1) {
    if (P->opt.local_prec >= 2) {
      const double m = (double)P->dh.m;
      w = 2.0 * m * m * P->nsub;
    } else {
      for (auto& t : P->types) w += 4.0 * t.box.nch * (double)t.box.b * t.box.b * t.nmem;
    }
  }
  Red dot = slot(P, 8);
  XrArgs xoff{};
  xoff.on = 0;
  CheckArgs coff{};
  coff.on = 0;
  const int fused = fused_coarse(P) ? 1 : 0;
  auto launch = [&]() {
    if (which == 0) launch_stencil(P, P->tabAs, x, y, nullptr, nullptr, s);
    // as launched inside the preconditioner: with the coarse space riding in
    // the dense launches, the GEMM carries R_0 r (of the internal residual),
    // the correction A_0^{-1} c and the extension forms the coarse field
    else if (which == 1) launch_local_solves(P, nullptr, s, fused ? P->r : nullptr);
    else if (which == 2) precond_apply(P, const_cast<double*>(x), y, nullptr, nullptr);
    else if (which == 3) launch_restrict(P, const_cast<double*>(x), nullptr, xoff, nullptr, s);
    else if (which == 4) launch_extend(P, x, y, P->opt.coarse, &dot, nullptr, coff, s, 0, fused);
    else if (P->opt.local_prec >= 2) launch_embed_fix(P, nullptr, s, fused);
  };
  launch();
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "event");
  check_hip(hipEventCreate(&e1), "event");
  check_hip(hipEventRecord(e0, s), "record");
  for (int i = 0; i < reps; ++i) launch();
  check_hip(hipEventRecord(e1, s), "record");
  check_hip(hipEventSynchronize(e1), "event sync");
  float ms = 0.0f;
  check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  check_launch("profile kernel");
  *avg_us = 1000.0 * ms / reps;
  if (work) *work = w;
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_profile_iteration(ddeig_problem* P, const double* b, int reps, double* us) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(b, "b")) return DDEIG_EINVAL;
  if (!us || reps < 1 || reps > 200) return set_error(DDEIG_EINVAL, "need us and 1 <= reps <= 200");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "profile_iteration before the shift is set");
  if (b == P->u) return set_error(DDEIG_EINVAL, "b must not be an internal vector");
  API_GUARD_BEGIN
  const hipStream_t s = P->stream;
  const long n = P->g.n;
  double* x = P->u;
  Red g = slot(P, 0), rr = slot(P, 1), rz = slot(P, 2);
  // a CG on A_sigma x = b from x = 0 that cannot stop: rtol 0 and maxit beyond
  // the iterations run, so no kernel takes its early exit
  const int maxit = reps + 2;
  launch_fill(x, n, 0.0, s);
  launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
  launch_resid_init(P, b, P->q, P->r, rr, s);
  launch_pcg_init(P, 0.0, rr, s);
  precond_apply(P, P->r, P->z, &rz, P->st);
  check_launch("profile start");
  const int coarse = P->opt.coarse;
  const bool fused = coarse && fused_coarse(P);
  constexpr int kParts = 5;
  std::vector<hipEvent_t> ev((size_t)(kParts + 1) * (reps + 1), nullptr);
  for (auto& e : ev) check_hip(hipEventCreate(&e), "event");
  for (int kk = 1; kk <= reps + 1; ++kk) {
    hipEvent_t* e = ev.data() + (size_t)(kParts + 1) * (kk - 1);
    double* pold = P->pp[(kk - 1) & 1];
    double* pnew = P->pp[kk & 1];
    const DirArgs dir{P->st, kk, rz};
    check_hip(hipEventRecord(e[0], s), "record");
    launch_stencil_dir(P, P->z, pold, pnew, P->q, dir, g, s);
    check_hip(hipEventRecord(e[1], s), "record");
    const XrArgs xr{1, kk, g, x, pnew, P->q};
    launch_restrict(P, P->r, P->st, xr, &rr, s);
    check_hip(hipEventRecord(e[2], s), "record");
    CheckArgs chk{1, kk, maxit, P->hist_cap, rr, P->hist};
    if (fused) {
      launch_local_solves(P, P->st, s, P->r);
      check_hip(hipEventRecord(e[3], s), "record");
      launch_embed_fix(P, P->st, s, true);
      check_hip(hipEventRecord(e[4], s), "record");
      launch_extend(P, P->r, P->z, 1, &rz, P->st, chk, s, 0, 1);
    } else {
      if (coarse) {
        check_hip(hipEventRecord(P->ev_fork, s), "record fork");
        check_hip(hipStreamWaitEvent(P->aux, P->ev_fork, 0), "wait fork");
      }
      launch_local_solves(P, P->st, s);
      check_hip(hipEventRecord(e[3], s), "record");
      if (P->opt.local_prec >= 2) launch_embed_fix(P, P->st, s);
      if (coarse) {
        launch_coarse_rhs(P, P->r, P->st, P->aux);
        launch_coarse_solve(P, P->st, P->aux);
        if (P->opt.local_prec >= 2) launch_coarse_field(P, P->st, P->aux);
        check_hip(hipEventRecord(P->ev_join, P->aux), "record join");
      }
      check_hip(hipEventRecord(e[4], s), "record");
      if (coarse) check_hip(hipStreamWaitEvent(s, P->ev_join, 0), "wait join");
      launch_extend(P, P->r, P->z, coarse, &rz, P->st, chk, s, 0);
    }
    check_hip(hipEventRecord(e[5], s), "record");
  }
  check_launch("profile iteration");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  for (int k = 0; k < kParts; ++k) us[k] = 0.0;
  for (int kk = 2; kk <= reps + 1; ++kk) {  // the first iteration is a warm-up
    hipEvent_t* e = ev.data() + (size_t)(kParts + 1) * (kk - 1);
    for (int k = 0; k < kParts; ++k) {
      float ms = 0.0f;
      check_hip(hipEventElapsedTime(&ms, e[k], e[k + 1]), "elapsed");
      us[k] += 1000.0 * ms / reps;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  PcgState hs{};
  check_hip(hipMemcpy(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost), "state");
  if (hs.done != 0)
    return set_error(DDEIG_EINTERNAL, "the profiled CG stopped early (state " +
                                          std::to_string(hs.done) + "); times are not valid");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_potential_form(ddeig_problem* P, int space, const ddeig_potential* W,
                                  const double* x, const double* y, double* out) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (!W || !out) return set_error(DDEIG_EINVAL, "potential or out is NULL");
  if (space != 0 && space != 1) return set_error(DDEIG_EINVAL, "space must be 0 or 1");
  if (validate_vec(x, "x") || validate_vec(y, "y")) return DDEIG_EINVAL;
  ddeig::VSpec ws{};
  {
    const ddeig_status sv = make_vspec(W, P->g.p, P->g.q, P->g.ell, ws);
    if (sv != DDEIG_OK) return sv;
    const ddeig_status st = check_quad_table(W, quad_table_len(P->g.p, P->g.q, P->g.ne, P->g.ell));
    if (st != DDEIG_OK) return st;
  }
  API_GUARD_BEGIN
  const hipStream_t s = P->stream;
  if (W->kind == DDEIG_V_QUAD_TABLE) {
    if (W->table_len > P->wtab_cap) {
      dfree(P, P->dWtab);
      P->dWtab = nullptr;
      P->wtab_cap = 0;
      P->dWtab = dalloc<double>(P, (size_t)W->table_len);
      P->wtab_cap = W->table_len;
    }
    sync(P);  // an earlier form may still read the table
    check_hip(hipMemcpy(P->dWtab, W->table, sizeof(double) * W->table_len,
                        hipMemcpyHostToDevice), "copy weight table");
    ws.table = P->dWtab;
  }
  check_hip(hipMemcpyAsync(P->dWS, &ws, sizeof(ddeig::VSpec), hipMemcpyHostToDevice, s), "copy W");
  launch_build_wtable(P, P->dWS, P->tabW, s);
  long len;
  if (space == 0) {
    launch_stencil(P, P->tabW, y, P->tmpv, nullptr, nullptr, s);
    len = P->g.n;
  } else {
    launch_box_stencil(P, cell_box(P->g), P->tabW, y, P->tmpv, nullptr, nullptr, s);
    len = P->g.tsize;
  }
  Red r = slot(P, 9);
  launch_dot(x, P->tmpv, len, r, s);
  check_launch("potential form");
  *out = host_sum(P, r);
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_potential_form_noalloc(ddeig_problem* P, int space, const ddeig_potential* W,
                                          const double* x, const double* y, double* out) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (!W || !out) return set_error(DDEIG_EINVAL, "potential or out is NULL");
  if (space != 0 && space != 1) return set_error(DDEIG_EINVAL, "space must be 0 or 1");
  if (validate_vec(x, "x") || validate_vec(y, "y")) return DDEIG_EINVAL;
  ddeig::VSpec ws{};
  {
    const ddeig_status sv = make_vspec(W, P->g.p, P->g.q, P->g.ell, ws);
    if (sv != DDEIG_OK) return sv;
    const ddeig_status st = check_quad_table(W, quad_table_len(P->g.p, P->g.q, P->g.ne, P->g.ell));
    if (st != DDEIG_OK) return st;
  }
  API_GUARD_BEGIN
  std::string err;
  const bool tab = W->kind == DDEIG_V_QUAD_TABLE;
  const ddeig_status st = ddeig::noalloc_form_checked(P, space, ws, tab ? W->table : nullptr,
                                                      tab ? W->table_len : 0, x, y, out, err);
  if (st != DDEIG_OK) return set_error(st, err);
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_eig_grad(ddeig_problem* P, const double* x, double* grad, int ngrad) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(x, "x")) return DDEIG_EINVAL;
  if (!grad) return set_error(DDEIG_EINVAL, "grad is NULL");
  int T = 0;
  if (grad_params(P, ngrad, T) != DDEIG_OK) return DDEIG_EINVAL;
  API_GUARD_BEGIN
  std::vector<GradJob> jobs{grad_job(P, x, x, 0)};
  std::vector<double> f;
  grad_run(P->allocs, P->gb, jobs, T, P->stream, f);
  if (!(f[2 * T] > 0.0)) return set_error(DDEIG_EINVAL, "x^T M x is not positive");
  for (int j = 0; j < 2 * T; ++j) grad[j] = f[j] / f[2 * T];
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_shift_grad(ddeig_problem* P, double* grad, int ngrad) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (!grad) return set_error(DDEIG_EINVAL, "grad is NULL");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "shift_grad before the shift is set");
  int T = 0;
  if (grad_params(P, ngrad, T) != DDEIG_OK) return DDEIG_EINVAL;
  API_GUARD_BEGIN
  std::vector<GradJob> jobs{grad_job(P, P->psi, P->psi, 1)};
  std::vector<double> f;
  grad_run(P->allocs, P->gb, jobs, T, P->stream, f);
  if (!(f[2 * T] > 0.0))
    return set_error(DDEIG_ESTATE, "no cell eigenvector (set_shift without psi)");
  for (int j = 0; j < 2 * T; ++j) grad[j] = f[j] / f[2 * T];
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_solve_grad(ddeig_problem* P, const double* u, const double* w, double* grad,
                              int ngrad) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(u, "u") || validate_vec(w, "w")) return DDEIG_EINVAL;
  if (!grad) return set_error(DDEIG_EINVAL, "grad is NULL");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "solve_grad before the shift is set");
  int T = 0;
  if (grad_params(P, ngrad, T) != DDEIG_OK) return DDEIG_EINVAL;
  API_GUARD_BEGIN
  std::vector<GradJob> jobs{grad_job(P, P->psi, P->psi, 1), grad_job(P, w, u, 0)};
  std::vector<double> f;
  grad_run(P->allocs, P->gb, jobs, T, P->stream, f);
  const int nf = 2 * T + 1;
  if (!(f[2 * T] > 0.0))
    return set_error(DDEIG_ESTATE, "no cell eigenvector (set_shift without psi)");
  for (int j = 0; j < 2 * T; ++j) {
    const double dsigma = f[j] / f[2 * T];
    grad[j] = -(f[nf + j] - dsigma * f[nf + 2 * T]);
  }
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_query(const ddeig_problem* P, long* n_dof, long* n_cell, int* n_sub) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (n_dof) *n_dof = P->g.n;
  if (n_cell) *n_cell = P->g.tsize;
  if (n_sub) *n_sub = P->nsub;
  return DDEIG_OK;
}

ddeig_status ddeig_set_shift(ddeig_problem* P, double sigma, const double* psi_cell_host) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (!std::isfinite(sigma)) return set_error(DDEIG_EINVAL, "sigma must be finite");
  if (psi_cell_host == nullptr && P->opt.coarse)
    return set_error(DDEIG_EINVAL, "the two-level preconditioner needs the cell vector psi");
  API_GUARD_BEGIN
  const auto t_start = std::chrono::steady_clock::now();
  P->shifted = 0;
  P->sigma = sigma;
  if (psi_cell_host)
    check_hip(hipMemcpyAsync(P->psi, psi_cell_host, sizeof(double) * P->g.tsize,
                             hipMemcpyHostToDevice, P->stream), "copy psi");
  sync(P);
  const ddeig_status st = finish_shift(P);
  P->t_setup_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                             t_start).count();
  return st;
  API_GUARD_END
}

ddeig_status ddeig_debug_force_breakdown(ddeig_problem* P, int count) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (count < 0) return set_error(DDEIG_EINVAL, "count must be >= 0");
  P->force_rz = count;
  return DDEIG_OK;
}

ddeig_status ddeig_cell_shift(ddeig_problem* P, double* sigma_out, double* psi_cell_host) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  API_GUARD_BEGIN
  const auto t_start = std::chrono::steady_clock::now();
  P->shifted = 0;
  const Geo& g = P->g;
  const hipStream_t s = P->stream;
  const Box cb = cell_box(g);
  const long nc = g.tsize;
  // a guaranteed lower bound of sigma: the stiffness in every fixed direction is
  // at least mu_min times the mass, the x parts are non-negative, and the
  // 2-point rule integrates the mass exactly, so M_V >= min V M
  double s0 = cell_vmin(P) - 1.0;
  for (int a = 0; a < g.D; ++a)
    if (!g.isx[a]) s0 += mu_min(g.nel[a], g.h);
  P->sigma = s0;
  launch_shift_table(P, s);
  double* Wc = dalloc<double>(P, (size_t)cb.nch * cb.b * cb.b);
  double* v0 = dalloc<double>(P, nc);  // psi_k
  double* v1 = dalloc<double>(P, nc);  // M psi_k
  double* v2 = dalloc<double>(P, nc);  // solve
  double* v3 = dalloc<double>(P, nc);  // M solve
  clear_flag(P);
  chain_factor(P, cb, P->tabAs, Wc, s);
  check_launch("cell factorisation");
  if (read_flag(P)) {
    dfree(P, Wc); dfree(P, v0); dfree(P, v1); dfree(P, v2); dfree(P, v3);
    return set_error(DDEIG_ENOTSPD, "cell operator shifted below its spectrum is not positive definite");
  }
  launch_fill(v0, nc, 1.0, s);
  double prev = INFINITY;
  int it = 0;
  for (; it < 2000; ++it) {
    launch_box_stencil(P, cb, P->tabM, v0, v1, nullptr, nullptr, s);
    launch_copy(v2, v1, nc, s);
    launch_chain_solve_box(P, cb, P->tabAs, Wc, v2, 1, s);
    Red s4 = slot(P, 4), s5 = slot(P, 5), s6 = slot(P, 6);
    launch_box_stencil(P, cb, P->tabM, v2, v3, &s4, &s5, s);
    launch_ipm_normalise(nc, v2, v3, v0, v1, s4, s5, s6, s);
    check_launch("cell iteration");
    const double d2 = host_sum(P, s6);
    const double d = std::sqrt(std::max(d2, 0.0));
    if (d <= 1e-14) break;
    if (it > 10 && d < 1e-12 && d > 0.8 * prev) break;  // stagnated at rounding level
    prev = d;
  }
  // sigma = psi^T A# psi with psi M#-normalised
  Red s4 = slot(P, 4);
  launch_box_stencil(P, cb, P->tabA, v0, v1, &s4, nullptr, s);
  const double sig = host_sum(P, s4);
  launch_copy(P->psi, v0, nc, s);
  if (psi_cell_host)
    check_hip(hipMemcpyAsync(psi_cell_host, v0, sizeof(double) * nc, hipMemcpyDeviceToHost, s), "copy psi");
  sync(P);
  dfree(P, Wc); dfree(P, v0); dfree(P, v1); dfree(P, v2); dfree(P, v3);
  P->sigma = sig;
  if (sigma_out) *sigma_out = sig;
  const ddeig_status st = finish_shift(P);
  P->t_setup_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                             t_start).count();
  return st;
  API_GUARD_END
}

ddeig_status ddeig_apply_op(ddeig_problem* P, int which, const double* x, double* y) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(x, "x") || validate_vec(y, "y")) return DDEIG_EINVAL;
  if (x == y) return set_error(DDEIG_EINVAL, "x and y must not alias");
  const double* tab = nullptr;
  switch (which) {
    case 0:
      if (!P->shifted) return set_error(DDEIG_ESTATE, "apply_op(A_sigma) before the shift is set");
      tab = P->tabAs;
      break;
    case 1: tab = P->tabA; break;
    case 2: tab = P->tabM; break;
    case 3: tab = P->tabK; break;
    default: return set_error(DDEIG_EINVAL, "which must be 0..3");
  }
  API_GUARD_BEGIN
  launch_stencil(P, tab, x, y, nullptr, nullptr, P->stream);
  check_launch("apply_op");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_apply_precond(ddeig_problem* P, const double* r, double* z) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(r, "r") || validate_vec(z, "z")) return DDEIG_EINVAL;
  if (r == z) return set_error(DDEIG_EINVAL, "r and z must not alias");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "apply_precond before the shift is set");
  API_GUARD_BEGIN
  precond_apply(P, const_cast<double*>(r), z, nullptr, nullptr);
  check_launch("apply_precond");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_apply_schwarz(ddeig_problem* P, int kind, const double* r, double* z) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(r, "r") || validate_vec(z, "z")) return DDEIG_EINVAL;
  if (r == z) return set_error(DDEIG_EINVAL, "r and z must not alias");
  const int flags = prec_flags(kind);
  if (flags < 0) return set_error(DDEIG_EINVAL, "unknown preconditioner kind");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "apply_schwarz before the shift is set");
  if ((flags & kPrecCoarse) && !P->opt.coarse)
    return set_error(DDEIG_ESTATE, "the problem was assembled without the coarse space");
  API_GUARD_BEGIN
  precond_apply(P, const_cast<double*>(r), z, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                flags);
  check_launch("apply_schwarz");
  return DDEIG_OK;
  API_GUARD_END
}

}  // extern "C"

namespace ddeig {

// ||b - A_sigma x||_2 / ||r_0||_2 recomputed from x (r_0 of the solve that
// left its state in P->st; 0 when r_0 = 0).
double true_relres(ddeig_problem* P, const double* b, const double* x) {
  const hipStream_t s = P->stream;
  Red rr = slot(P, 10);
  launch_stencil(P, P->tabAs, x, P->q, nullptr, nullptr, s);
  launch_resid_init(P, b, P->q, P->r, rr, s);
  const double rn2 = host_sum(P, rr);
  PcgState hs{};
  check_hip(hipMemcpy(&hs, P->st, sizeof(PcgState), hipMemcpyDeviceToHost), "state");
  return hs.r0n2 > 0.0 ? std::sqrt(std::max(rn2, 0.0) / hs.r0n2) : 0.0;
}

// ||A x - lambda M x||_2 of an M-normalised x.
double spectral_residual(ddeig_problem* P, const double* x, double lambda) {
  const hipStream_t s = P->stream;
  launch_stencil(P, P->tabA, x, P->q, nullptr, nullptr, s);
  launch_stencil(P, P->tabM, x, P->z, nullptr, nullptr, s);
  Red rr = slot(P, 11);
  launch_lopcg_resid(P->g.n, lambda, P->q, P->z, P->w, rr.part, rr.val, s);
  double v = 0.0;
  check_hip(hipMemcpyAsync(&v, rr.val, sizeof(double), hipMemcpyDeviceToHost, s), "copy scalar");
  sync(P);
  return std::sqrt(std::max(v, 0.0));
}

}  // namespace ddeig

extern "C" {

static void fill_info(ddeig_problem* P, const PcgOut& o, int breakdown, ddeig_pcg_info* info,
                      const double* b = nullptr, const double* x = nullptr) {
  if (!info) return;
  info->iters = o.iters;
  info->relres = o.relres;
  info->breakdown = breakdown;
  info->fallback = 0;
  info->true_relres = b ? ddeig::true_relres(P, b, x) : o.relres;
  if (info->hist && info->hist_cap > 0) {
    const int cnt = std::min(std::min(info->hist_cap, o.iters + 1), P->hist_cap);
    check_hip(hipMemcpyAsync(info->hist, P->hist, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                             P->stream), "copy history");
    sync(P);
  }
}

ddeig_status ddeig_stationary_ras(ddeig_problem* P, int levels, const double* b, double* x,
                                  double rtol, int maxit, ddeig_pcg_info* info) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(b, "b") || validate_vec(x, "x")) return DDEIG_EINVAL;
  if (b == x) return set_error(DDEIG_EINVAL, "b and x must not alias");
  if (levels != 1 && levels != 2) return set_error(DDEIG_EINVAL, "levels must be 1 or 2");
  if (!(rtol >= 0.0) || !std::isfinite(rtol) || maxit < 0)
    return set_error(DDEIG_EINVAL, "need rtol >= 0 and maxit >= 0");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "stationary_ras before the shift is set");
  if (levels == 2 && !P->opt.coarse)
    return set_error(DDEIG_ESTATE, "the problem was assembled without the coarse space");
  API_GUARD_BEGIN
  const PcgOut o = sras_run(P, levels, b, x, rtol, maxit);
  fill_info(P, o, o.done == 2 ? 1 : 0, info, b, x);
  if (o.done == 2) return set_error(DDEIG_ENOCONV, "stationary RAS diverged");
  if (o.done != 1) return set_error(DDEIG_ENOCONV, "stationary RAS reached maxit");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_gmres_solve(ddeig_problem* P, int kind, const double* b, double* x, double rtol,
                               int maxit, int restart, ddeig_pcg_info* info) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(b, "b") || validate_vec(x, "x")) return DDEIG_EINVAL;
  if (b == x) return set_error(DDEIG_EINVAL, "b and x must not alias");
  const int flags = prec_flags(kind);
  if (flags < 0) return set_error(DDEIG_EINVAL, "unknown preconditioner kind");
  if (!(rtol >= 0.0) || !std::isfinite(rtol) || maxit < 0)
    return set_error(DDEIG_EINVAL, "need rtol >= 0 and maxit >= 0");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "gmres_solve before the shift is set");
  if ((flags & kPrecCoarse) && !P->opt.coarse)
    return set_error(DDEIG_ESTATE, "the problem was assembled without the coarse space");
  API_GUARD_BEGIN
  const int m = std::min(kGmMaxRestart,
                         std::max(1, restart > 0 ? std::min(restart, std::max(maxit, 1))
                                                 : std::min(std::max(maxit, 1), 300)));
  const PcgOut o = gmres_run(P, flags, b, x, rtol, maxit, m);
  fill_info(P, o, o.done == 2 ? 1 : 0, info, b, x);
  if (o.done == 2) return set_error(DDEIG_ENOCONV, "GMRES breakdown (zero Hessenberg column)");
  if (o.done != 1) return set_error(DDEIG_ENOCONV, "GMRES reached maxit");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_pcg_solve(ddeig_problem* P, const double* b, double* x, double rtol, int maxit,
                             ddeig_pcg_info* info) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(b, "b") || validate_vec(x, "x")) return DDEIG_EINVAL;
  if (b == x) return set_error(DDEIG_EINVAL, "b and x must not alias");
  if (!(rtol >= 0.0) || !std::isfinite(rtol) || maxit < 0)
    return set_error(DDEIG_EINVAL, "need rtol >= 0 and maxit >= 0");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "pcg_solve before the shift is set");
  API_GUARD_BEGIN
  const int fb0 = P->fallbacks;
  const bool can_fall_back = P->opt.local_prec >= 2 && P->g.D == 2;
  if (can_fall_back) launch_copy(P->tmpv, x, P->g.n, P->stream);  // x0, for a repeat
  PcgOut o = pcg_run(P, b, x, rtol, maxit);
  if (o.done == 3 && can_fall_back && fallback_fp32(P)) {
    launch_copy(x, P->tmpv, P->g.n, P->stream);
    o = pcg_run(P, b, x, rtol, maxit);
  }
  fill_info(P, o, o.done == 2 ? 1 : (o.done == 3 ? 2 : 0), info, b, x);
  if (info) info->fallback = P->fallbacks - fb0;
  if (o.done == 2 || o.done == 3)
    return set_error(DDEIG_ENOTSPD, o.done == 2 ? "CG breakdown: p.A_sigma p <= 0"
                                                : "CG breakdown: r.z <= 0");
  if (o.done != 1) return set_error(DDEIG_ENOCONV, "PCG reached maxit");
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_inverse_iteration(ddeig_problem* P, double* x, double tol_x, int maxit_outer,
                                     double rtol_inner, int maxit_inner, ddeig_eig_info* info) {
  if (!P) return set_error(DDEIG_EINVAL, "problem is NULL");
  if (validate_vec(x, "x")) return DDEIG_EINVAL;
  if (!(tol_x >= 0.0) || maxit_outer < 1 || !(rtol_inner >= 0.0) || maxit_inner < 1)
    return set_error(DDEIG_EINVAL, "invalid tolerances or iteration limits");
  if (!P->shifted) return set_error(DDEIG_ESTATE, "inverse_iteration before the shift is set");
  API_GUARD_BEGIN
  const hipStream_t s = P->stream;
  const long n = P->g.n;
  const auto t0 = std::chrono::steady_clock::now();
  // start vector: x, or 1/||1||_M if x is all zeros
  Red s3 = slot(P, 3);
  launch_dot(x, x, n, s3, s);
  if (host_sum(P, s3) == 0.0) {
    launch_fill(P->u, n, 1.0, s);
    launch_stencil(P, P->tabM, P->u, P->w, &s3, nullptr, s);
    launch_scale_copy(n, x, P->u, s3, s);
  }
  double lam = 0.0, dx = INFINITY;
  long inner_sum = 0;
  int inner_max = 0, k = 0, inner_unconv = 0;
  ddeig_status st = DDEIG_ENOCONV;
  const int fb0 = P->fallbacks;
  for (k = 1; k <= maxit_outer; ++k) {
    launch_stencil(P, P->tabM, x, P->w, nullptr, nullptr, s);  // b = M x
    launch_fill(P->u, n, 0.0, s);
    PcgOut o = pcg_run(P, P->w, P->u, rtol_inner, maxit_inner);
    if (o.done == 3 && fallback_fp32(P)) {
      launch_fill(P->u, n, 0.0, s);
      o = pcg_run(P, P->w, P->u, rtol_inner, maxit_inner);
    }
    if (o.done == 2 || o.done == 3) {
      st = set_error(DDEIG_ENOTSPD, "CG breakdown inside inverse iteration");
      break;
    }
    inner_sum += o.iters;
    inner_max = std::max(inner_max, o.iters);
    if (o.done != 1) ++inner_unconv;  // stopped at maxit_inner
    Red s4 = slot(P, 4), s5 = slot(P, 5), s6 = slot(P, 6), s7 = slot(P, 7);
    launch_stencil(P, P->tabM, P->u, P->z, &s4, &s5, s);  // Mu, u.Mu, sum(Mu)
    launch_ipm_normalise(n, P->u, P->z, x, P->w, s4, s5, s6, s);
    launch_stencil(P, P->tabAs, x, P->q, &s7, nullptr, s);  // x.A_sigma x
    launch_finish_sum(s6, s);
    launch_finish_sum(s7, s);
    double hs[2];
    check_hip(hipMemcpyAsync(hs, P->red_val + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
              "copy");
    sync(P);
    dx = std::sqrt(std::max(hs[0], 0.0));
    lam = P->sigma + hs[1];
    if (dx <= tol_x) {
      st = DDEIG_OK;
      break;
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->lambda = lam;
    info->dx_M = dx;
    info->outer_its = std::min(k, maxit_outer);
    info->inner_sum = inner_sum;
    info->inner_max = inner_max;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    info->spec_res = ddeig::spectral_residual(P, x, lam);
    info->t_setup_ms = P->t_setup_ms;
    info->inner_unconverged = inner_unconv;
    info->fallback = P->fallbacks - fb0;
  }
  if (st == DDEIG_ENOCONV) return set_error(st, "inverse iteration reached maxit_outer");
  // an inner solve that stopped at maxit_inner can leave the outer test on the
  // fixed point of the inexact solve, so the pair is not reported as converged
  if (st == DDEIG_OK && inner_unconv > 0)
    return set_error(DDEIG_ENOCONV, std::to_string(inner_unconv) +
                                        " inner solve(s) stopped at maxit_inner");
  return st;
  API_GUARD_END
}

}  // extern "C"

// ---- batches of independent problems ---------------------------------------
//
// Instances that share the mesh width, the overlap, the fixed-direction
// extent and the dense local-solve mode (2-D, one expanding axis) have dense
// boxes of one shape, so every kernel of a PCG iteration can run as one
// grouped launch over all of them: a block map sends each block to (instance,
// block within the instance), the MFMA tiles and the clipped-class jobs carry
// their instance, and every instance keeps its own CG scalars, partial sums
// and stopping test (its `done` flag turns its blocks into no-ops).  The
// start of each solve and the inverse-iteration normalisation run per
// instance.

struct ddeig_batch {
  std::vector<ddeig_problem*> P;
  hipStream_t stream = nullptr, aux = nullptr, cap = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int n = 0, local_prec = 0, ksplit = 1, order = 0;
  int ld = 0, hm0 = 0, hm1 = 0, mH = 0;
  std::vector<ddeig::InstDev> inst;
  ddeig::InstDev* dInst = nullptr;
  ddeig::BlockMap bm_st{}, bm_node{}, bm_crhs{}, bm_csol{}, bm_cf{};
  ddeig::GemmTile* dTiles = nullptr;
  int ntiles = 0;
  ddeig::GemmType* dGt = nullptr;
  ddeig::EmbedJob* dEmbJobs = nullptr;
  int nembjobs = 0;
  ddeig::EmbedDev* dEmb = nullptr;
  ddeig::PcgState* dStates = nullptr;
  std::vector<ddeig::PcgState> hStates;
  double* dRes = nullptr;
  int* dAct = nullptr;   // 2 n activity flags of the grouped outer-iteration launches
  int* hAct = nullptr;   // pinned host copy
  ddeig::PcgState* hst = nullptr;             // pinned: CG states behind two blocks of iterations
  hipEvent_t ev_st[2] = {nullptr, nullptr};   // recorded after each block's state copy
  std::vector<void*> allocs;
  int tile_rows = 128;      // GEMM tile rows (128, or 64 to skip padding rows)
  double tune_us[12] = {};  // [tile rows 128, 64][split 1..3][order 0..1]
  // hipGraph replay of the grouped iterations: one executable graph per
  // (first iteration of a block of 8, maxit), captured on first use
  int use_graphs = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  ddeig::GradBuf gb;  // derivative forms of ddeig_batch_eig_grad / ddeig_batch_solve_grad
};

namespace {

// GEMM choices of the batch autotuner by shape, for the life of the process
std::mutex g_tune_mu;
std::map<std::string, std::array<int, 3>> g_tune;

template <typename T>
T* balloc(ddeig_batch* B, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    throw Failure{DDEIG_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
  }
  B->allocs.push_back(p);
  return static_cast<T*>(p);
}

template <typename T>
T* bupload(ddeig_batch* B, const std::vector<T>& v) {
  T* d = balloc<T>(B, v.size());
  check_hip(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice), "batch upload");
  return d;
}

ddeig::BlockMap make_map(ddeig_batch* B, const std::vector<int>& counts) {
  std::vector<int2> m;
  for (size_t j = 0; j < counts.size(); ++j)
    for (int b = 0; b < counts[j]; ++b) m.push_back(make_int2((int)j, b));
  return ddeig::BlockMap{bupload(B, m), (int)m.size()};
}

// MFMA tiles of every instance for a K split of ks: a group is the row tiles
// of one (instance, column tile, split), which read the same rows of that
// instance's inverse.  order 1 interleaves eight groups of equal size so that
// a group's tiles get workgroup ids 8 apart (one XCD, one L2 copy of the rows).
std::vector<ddeig::GemmTile> batch_tiles(const ddeig_batch* B, int ks, int order, int tm) {
  const int bk = B->local_prec == 2 ? 32 : 64;
  const int npair = B->ld / bk / 2;
  std::vector<std::vector<ddeig::GemmTile>> groups;
  for (int j = 0; j < B->n; ++j) {
    // row tiles of tm rows covering the instance's subdomains (the rows past
    // them, up to its padded row count, are skipped when tm = 64)
    const int nrt = (B->P[j]->nsub + tm - 1) / tm;
    for (int sp = 0; sp < ks; ++sp) {
      const int kb0 = 2 * (int)((long)npair * sp / ks);
      const int kb1 = 2 * (int)((long)npair * (sp + 1) / ks);
      for (int nt = 0; nt < B->ld / 128; ++nt) {
        std::vector<ddeig::GemmTile> grp;
        for (int mt = 0; mt < nrt; ++mt)
          grp.push_back(ddeig::GemmTile{j, mt * tm, nt * 128, kb0 * bk, kb1 * bk, sp});
        groups.push_back(grp);
      }
    }
  }
  std::vector<ddeig::GemmTile> tiles;
  if (order == 0) {
    for (auto& g : groups)
      for (auto& t : g) tiles.push_back(t);
    return tiles;
  }
  std::stable_sort(groups.begin(), groups.end(),
                   [](const std::vector<ddeig::GemmTile>& a, const std::vector<ddeig::GemmTile>& b) {
                     return a.size() > b.size();
                   });
  size_t gi = 0;
  while (gi < groups.size()) {
    size_t gj = gi;
    while (gj < groups.size() && gj - gi < 8 && groups[gj].size() == groups[gi].size()) ++gj;
    for (size_t i = 0; i < groups[gi].size(); ++i)
      for (size_t j = gi; j < gj; ++j) tiles.push_back(groups[j][i]);
    gi = gj;
  }
  return tiles;
}

void batch_upload_inst(ddeig_batch* B) {
  check_hip(hipMemcpyAsync(B->dInst, B->inst.data(), sizeof(ddeig::InstDev) * B->n,
                           hipMemcpyHostToDevice, B->stream), "upload instances");
  check_hip(hipStreamSynchronize(B->stream), "hipStreamSynchronize");
}

// One grouped PCG iteration k over every instance (see pcg_run for the kernels),
// issued on stream s (the batch's stream, or its capture stream).
void batch_iteration(ddeig_batch* B, int k, int maxit, hipStream_t s) {
  launch_b_stencil_dir(B->dInst, B->bm_st, k, s);
  launch_b_restrict(B->dInst, B->bm_node, k, s);
  check_hip(hipEventRecord(B->ev_fork, s), "record fork");
  check_hip(hipStreamWaitEvent(B->aux, B->ev_fork, 0), "wait fork");
  launch_gemm_tiles(B->dTiles, B->ntiles, B->dGt, B->local_prec, s, B->tile_rows);
  launch_embed_jobs(B->dEmbJobs, B->nembjobs, B->dEmb, B->ksplit, B->ld, B->hm0, B->hm1, B->mH, s);
  launch_b_coarse_rhs(B->dInst, B->bm_crhs, B->aux);
  launch_b_coarse_solve(B->dInst, B->bm_csol, B->aux);
  launch_b_coarse_field(B->dInst, B->bm_cf, B->aux);
  check_hip(hipEventRecord(B->ev_join, B->aux), "record join");
  check_hip(hipStreamWaitEvent(s, B->ev_join, 0), "wait join");
  launch_b_extend(B->dInst, B->bm_node, k, maxit, B->ksplit, s);
}

// PCG on A_sigma,j x_j = b_j for the instances with active[j] != 0 (the
// others stay idle); on return B->hStates holds every instance's final state.
// With act (device flags of the active instances, already on the stream) the
// start is grouped: x_0 = 0 and b = the instance's w, as in the inverse
// iteration; otherwise each instance starts from its own x_0 and b.
void batch_pcg(ddeig_batch* B, const std::vector<int>& active, const std::vector<const double*>& b,
               const std::vector<double*>& x, double rtol, int maxit, const int* act = nullptr) {
  const hipStream_t s = B->stream;
  for (int j = 0; j < B->n; ++j) B->inst[j].x = x[j];
  batch_upload_inst(B);
  launch_b_states(B->dInst, B->n, B->dStates, 1, s);
  if (act != nullptr) {
    launch_b_restrict_start(B->dInst, B->bm_node, act, s);
    launch_b_pcg_init(B->dInst, B->n, act, rtol, s);
    check_hip(hipEventRecord(B->ev_fork, s), "record fork");
    check_hip(hipStreamWaitEvent(B->aux, B->ev_fork, 0), "wait fork");
    launch_gemm_tiles(B->dTiles, B->ntiles, B->dGt, B->local_prec, s, B->tile_rows);
    launch_embed_jobs(B->dEmbJobs, B->nembjobs, B->dEmb, B->ksplit, B->ld, B->hm0, B->hm1, B->mH,
                      s);
    launch_b_coarse_rhs(B->dInst, B->bm_crhs, B->aux);
    launch_b_coarse_solve(B->dInst, B->bm_csol, B->aux);
    launch_b_coarse_field(B->dInst, B->bm_cf, B->aux);
    check_hip(hipEventRecord(B->ev_join, B->aux), "record join");
    check_hip(hipStreamWaitEvent(s, B->ev_join, 0), "wait join");
    launch_b_extend(B->dInst, B->bm_node, 0, maxit, B->ksplit, s, 0);
  } else {
    for (int j = 0; j < B->n; ++j) {
      if (!active[j]) continue;
      ddeig_problem* P = B->P[j];
      Red rr = slot(P, 1), rz = slot(P, 2);
      launch_stencil(P, P->tabAs, x[j], P->q, nullptr, nullptr, s);
      launch_resid_init(P, b[j], P->q, P->r, rr, s);
      launch_pcg_init(P, rtol, rr, s);
      precond_apply(P, P->r, P->z, &rz, P->st);
    }
  }
  check_launch("batch pcg start");
  // blocks of 8 iterations; the next block is queued before the host looks at
  // the states copied behind the current one (pinned slot sl), so the device
  // does not idle during the check (a block queued after every instance has
  // stopped is a no-op: its kernels see the final states)
  const int n = B->n;
  auto submit = [&](int k0, int kend, int sl) {
    if (B->use_graphs && kend >= k0) {
      const auto key = std::make_pair(k0, maxit);
      auto it = B->graphs.find(key);
      if (it == B->graphs.end()) {
        hipGraph_t gr = nullptr;
        hipGraphExec_t ge = nullptr;
        // captured on the batch's own stream (the problems' stream may be the
        // null stream, which cannot capture), launched on the problems' stream
        const hipStream_t cs = B->cap;
        check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
          for (int kk = k0; kk <= kend; ++kk) batch_iteration(B, kk, maxit, cs);
        } catch (...) {
          (void)hipStreamEndCapture(cs, &gr);
          if (gr) (void)hipGraphDestroy(gr);
          throw;
        }
        check_hip(hipStreamEndCapture(cs, &gr), "end capture");
        const hipError_t e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        check_hip(e, "instantiate graph");
        it = B->graphs.emplace(key, ge).first;
      }
      check_hip(hipGraphLaunch(it->second, s), "launch graph");
    } else {
      for (int kk = k0; kk <= kend; ++kk) batch_iteration(B, kk, maxit, s);
    }
    check_launch("batch pcg iteration");
    launch_b_states(B->dInst, n, B->dStates, 0, s);
    check_hip(hipMemcpyAsync(B->hst + (size_t)sl * n, B->dStates, sizeof(ddeig::PcgState) * n,
                             hipMemcpyDeviceToHost, s), "copy states");
    check_hip(hipEventRecord(B->ev_st[sl], s), "record states");
  };
  int k = std::min(maxit, 8), sl = 0;
  submit(1, k, 0);
  for (;;) {
    const bool more = k < maxit;
    const int knext = std::min(maxit, k + 8);
    if (more) submit(k + 1, knext, sl ^ 1);
    check_hip(hipEventSynchronize(B->ev_st[sl]), "wait states");
    std::copy(B->hst + (size_t)sl * n, B->hst + (size_t)(sl + 1) * n, B->hStates.begin());
    bool all_done = true;
    for (int j = 0; j < n; ++j)
      if (active[j] && B->hStates[j].done == 0) all_done = false;
    if (all_done || !more) break;
    k = knext;
    sl ^= 1;
  }
  // maxit reached without a stopping decision (maxit = 0 or a state still running)
  for (int j = 0; j < B->n; ++j)
    if (active[j] && B->hStates[j].done == 0) B->hStates[j].done = 4;
}

float time_gemm(ddeig_batch* B, const ddeig::GemmTile* dT, int nt, const ddeig::GemmType* gt,
                int tm) {
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "event");
  check_hip(hipEventCreate(&e1), "event");
  for (int i = 0; i < 3; ++i) launch_gemm_tiles(dT, nt, gt, B->local_prec, B->stream, tm);
  check_hip(hipEventRecord(e0, B->stream), "record");
  const int reps = 10;
  for (int i = 0; i < reps; ++i) launch_gemm_tiles(dT, nt, gt, B->local_prec, B->stream, tm);
  check_hip(hipEventRecord(e1, B->stream), "record");
  check_hip(hipEventSynchronize(e1), "sync");
  float ms = 0.0f;
  check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  check_launch("gemm tuning");
  return 1000.0f * ms / reps;
}

void batch_free(ddeig_batch* B) {
  if (!B) return;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  for (auto& kv : B->graphs) (void)hipGraphExecDestroy(kv.second);
  for (void* p : B->allocs) (void)hipFree(p);
  if (B->aux) (void)hipStreamDestroy(B->aux);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  if (B->ev_join) (void)hipEventDestroy(B->ev_join);
  if (B->hAct) (void)hipHostFree(B->hAct);
  if (B->hst) (void)hipHostFree(B->hst);
  for (auto& e : B->ev_st)
    if (e) (void)hipEventDestroy(e);
  delete B;
}

}  // namespace

extern "C" {

ddeig_status ddeig_batch_create(ddeig_problem* const* probs, int n, int flags, ddeig_batch** out) {
  if (!probs || !out) return set_error(DDEIG_EINVAL, "probs or out is NULL");
  *out = nullptr;
  if (n < 1 || n > 4096) return set_error(DDEIG_EINVAL, "need 1 <= n <= 4096 instances");
  if (flags & ~(DDEIG_BATCH_GRAPHS | DDEIG_BATCH_REPRODUCIBLE | DDEIG_BATCH_TILE64))
    return set_error(DDEIG_EINVAL, "unknown batch flags");
  if ((flags & DDEIG_BATCH_TILE64) && !(flags & DDEIG_BATCH_REPRODUCIBLE))
    return set_error(DDEIG_EINVAL, "DDEIG_BATCH_TILE64 needs DDEIG_BATCH_REPRODUCIBLE");
  const ddeig_problem* P0 = probs[0];
  for (int j = 0; j < n; ++j) {
    const ddeig_problem* P = probs[j];
    if (!P) return set_error(DDEIG_EINVAL, "instance " + std::to_string(j) + " is NULL");
    for (int i = 0; i < j; ++i)
      if (probs[i] == P) return set_error(DDEIG_EINVAL, "an instance appears twice");
    const std::string who = "instance " + std::to_string(j) + ": ";
    if (P->g.D != 2 || P->g.p != 1)
      return set_error(DDEIG_EINVAL, who + "batches need p = 1, q = 1 (2-D)");
    if (P->opt.local_prec < 2 || P->opt.coarse != 1)
      return set_error(DDEIG_EINVAL, who + "batches need dense local solves (local_prec 2 or 3) "
                                           "and the coarse space");
    if (64 % P->g.ne != 0) return set_error(DDEIG_EINVAL, who + "batches need n_e dividing 64");
    if (P->nsub <= ddeig::kGemvMax)
      return set_error(DDEIG_EINVAL, who + "batches need L > " + std::to_string(ddeig::kGemvMax));
    if (ddeig::stencil_tiles(P->g) > kMaxRed)
      return set_error(DDEIG_EINVAL, who + "instance too large for a batch (stencil tiles > 1024)");
    // the grouped GEMM reads R through buffer resources with 32-bit byte counts
    if ((long)P->dh.mp * P->dh.ld * 2 >= (1L << 31))
      return set_error(DDEIG_EINVAL, who + "instance too large for a batch (restricted residuals)");
    if (P->opt.local_prec != P0->opt.local_prec || P->g.ne != P0->g.ne ||
        P->delta != P0->delta || P->g.N[1] != P0->g.N[1] || P->dh.ld != P0->dh.ld ||
        P->dh.m != P0->dh.m || P->stream != P0->stream || P->opt.pu != P0->opt.pu)
      return set_error(DDEIG_EINVAL, who + "instances of a batch need the same n_e, overlap, ell, "
                                           "partition of unity, local_prec and stream");
  }
  ddeig_batch* B = nullptr;
  try {
    B = new ddeig_batch();
  } catch (const std::bad_alloc&) {
    return set_error(DDEIG_ENOMEM, "host allocation failed");
  }
  try {
    B->n = n;
    B->use_graphs = (flags & DDEIG_BATCH_GRAPHS) ? 1 : 0;
    B->P.assign(probs, probs + n);
    B->stream = P0->stream;
    B->local_prec = P0->opt.local_prec;
    B->ld = P0->dh.ld;
    B->hm0 = P0->dh.box.m[0];
    B->hm1 = P0->dh.box.m[1];
    B->mH = P0->dh.m;
    check_hip(hipStreamCreateWithFlags(&B->aux, hipStreamNonBlocking), "create batch stream");
    if (B->use_graphs)
      check_hip(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking), "create capture stream");
    check_hip(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming), "create event");
    check_hip(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming), "create event");
    int ks_max = 3;
    for (auto* P : B->P) ks_max = std::min(ks_max, P->ksplit);
    // grouped-GEMM tiles: a small autotuner times every K split the Z buffers
    // allow, with and without the XCD interleave, and keeps the fastest
    std::vector<ddeig::GemmType> gts(n), gtt(n);
    for (int j = 0; j < n; ++j) {
      const ddeig::DenseHost& H = B->P[j]->dh;
      gts[j] = ddeig::GemmType{H.Ah, H.Al, H.Rh, H.Rl, H.Z, (long)H.mp * H.ld, H.ld,
                               B->P[j]->nsub, B->P[j]->st};
      gtt[j] = gts[j];
      gtt[j].st = nullptr;
    }
    B->dGt = bupload(B, gts);
    std::vector<ddeig::GemmTile> best_tiles;
    std::string shape = std::to_string(B->local_prec) + "/" + std::to_string(B->ld) + "/" +
                        std::to_string(ks_max);
    for (auto* P : B->P) shape += "/" + std::to_string(P->nsub);
    std::array<int, 3> choice{0, 0, 0};  // K split, order, tile rows
    if (flags & DDEIG_BATCH_REPRODUCIBLE) {
      choice = {ks_max, 1, (flags & DDEIG_BATCH_TILE64) ? 64 : 128};
    } else {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(shape);
      if (it != g_tune.end()) choice = it->second;
    }
    if (choice[0] > 0) {
      B->ksplit = choice[0];
      B->order = choice[1];
      B->tile_rows = choice[2];
      best_tiles = batch_tiles(B, B->ksplit, B->order, B->tile_rows);
    } else {
      // every tile shape (128 or 64 rows), K split and order; the tile rows do
      // not change the arithmetic (each output sums the same K stages in the
      // same order), the K split does
      ddeig::GemmType* dGtt = bupload(B, gtt);
      float best = 1e30f;
      for (int ti = 0; ti < 2; ++ti) {
        const int tm = ti == 0 ? 128 : 64;
        for (int ks = 1; ks <= ks_max; ++ks)
          for (int order = 0; order < 2; ++order) {
            std::vector<ddeig::GemmTile> t = batch_tiles(B, ks, order, tm);
            ddeig::GemmTile* dT = bupload(B, t);
            const float us = time_gemm(B, dT, (int)t.size(), dGtt, tm);
            B->tune_us[ti * 6 + (ks - 1) * 2 + order] = us;
            if (us < best) {
              best = us;
              best_tiles = t;
              B->ksplit = ks;
              B->order = order;
              B->tile_rows = tm;
            }
          }
      }
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune.emplace(shape, std::array<int, 3>{B->ksplit, B->order, B->tile_rows});
    }
    B->dTiles = bupload(B, best_tiles);
    B->ntiles = (int)best_tiles.size();
    // clipped classes of every instance, each checked against its instance's state
    std::vector<ddeig::EmbedDev> emb;
    std::vector<ddeig::EmbedJob> jobs;
    for (int j = 0; j < n; ++j)
      for (const auto& E0 : B->P[j]->emb) {
        ddeig::EmbedDev E = E0;
        E.st = B->P[j]->st;
        const int ci2 = (int)emb.size();
        emb.push_back(E);
        const int per = ddeig::emb_members_per_job(E.nT);
        for (int m0 = 0; m0 < E.nmem; m0 += per)
          jobs.push_back(ddeig::EmbedJob{ci2, m0, std::min(per, E.nmem - m0)});
      }
    if (jobs.size() > (size_t)ddeig::kEmbMaxJobs)
      throw Failure{DDEIG_EINVAL, "batch: more than 65535 clipped-subdomain correction jobs; "
                                  "use fewer instances"};
    B->nembjobs = (int)jobs.size();
    if (!emb.empty()) {
      B->dEmb = bupload(B, emb);
      B->dEmbJobs = bupload(B, jobs);
    }
    // instance descriptors and block maps
    B->inst.resize(n);
    std::vector<int> c_st(n), c_node(n), c_crhs(n), c_csol(n), c_cf(n);
    for (int j = 0; j < n; ++j) {
      ddeig_problem* P = B->P[j];
      const ddeig::DenseHost& H = P->dh;
      ddeig::InstDev& d = B->inst[j];
      d.g = P->g;
      d.delta = P->delta;
      d.pu = P->opt.pu;
      d.nsub = P->nsub;
      d.nb_node = ddeig::node_grid_dense(P->g);  // the single problem's grid (2 nodes per thread)
      d.nb_cf = ddeig::coarse_field_grid(P->g);
      d.hist_cap = P->hist_cap;
      d.tabAs = P->tabAs;
      d.x = P->u;
      d.r = P->r;
      d.z = P->z;
      d.q = P->q;
      d.pp[0] = P->pp[0];
      d.pp[1] = P->pp[1];
      d.st = P->st;
      d.gam = slot(P, 0);
      d.gam.np = (int)ddeig::stencil_tiles(P->g);
      d.sty = ddeig::stencil2d_ty(P->g);
      d.rr = slot(P, 1);
      d.rr.np = d.nb_node;
      d.rz = slot(P, 2);
      d.rz.np = d.nb_node;
      d.da = ddeig::DenseArgs{H.Rh, H.Rl, H.Z, (long)H.mp * H.ld, H.ld, B->ksplit, H.box.m[0],
                              H.box.m[1]};
      d.psi = P->psi;
      d.cf = P->cfield;
      d.types = P->dTypes;
      d.subs = P->dSubs;
      d.crhs = P->crhs;
      d.A0inv = P->A0inv;
      d.cy = P->cy;
      d.xc0 = P->dXC[0];
      d.hist = P->hist;
      d.tabM = P->tabM;
      d.xo = nullptr;
      d.w = P->w;
      d.nm_uMu = slot(P, 4);
      d.nm_uMu.np = d.gam.np;
      d.nm_sum = slot(P, 5);
      d.nm_sum.np = d.gam.np;
      d.nm_dx = slot(P, 6);
      d.nm_dx.np = d.nb_node;
      d.nm_xq = slot(P, 7);
      d.nm_xq.np = d.gam.np;
      c_st[j] = d.gam.np;
      c_node[j] = d.nb_node;
      c_crhs[j] = P->nsub;
      c_csol[j] = (P->nsub + kBlock / 64 - 1) / (kBlock / 64);
      c_cf[j] = d.nb_cf;
    }
    B->dInst = balloc<ddeig::InstDev>(B, n);
    B->bm_st = make_map(B, c_st);
    B->bm_node = make_map(B, c_node);
    B->bm_crhs = make_map(B, c_crhs);
    B->bm_csol = make_map(B, c_csol);
    B->bm_cf = make_map(B, c_cf);
    B->dStates = balloc<ddeig::PcgState>(B, n);
    B->hStates.resize(n);
    B->dRes = balloc<double>(B, 2 * (size_t)n);
    B->dAct = balloc<int>(B, 2 * (size_t)n);
    check_hip(hipHostMalloc(reinterpret_cast<void**>(&B->hAct), 2 * (size_t)n * sizeof(int)),
              "hipHostMalloc");
    check_hip(hipHostMalloc(reinterpret_cast<void**>(&B->hst),
                            2 * (size_t)n * sizeof(ddeig::PcgState)), "hipHostMalloc");
    for (auto& e : B->ev_st)
      check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "create event");
    check_hip(hipStreamSynchronize(B->stream), "hipStreamSynchronize");
  } catch (const Failure& f) {
    batch_free(B);
    return set_error(f.status, f.msg);
  } catch (const std::bad_alloc&) {
    batch_free(B);
    return set_error(DDEIG_ENOMEM, "host allocation failed");
  } catch (...) {
    batch_free(B);
    return set_error(DDEIG_EINTERNAL, "unexpected internal exception");
  }
  *out = B;
  return DDEIG_OK;
}

ddeig_status ddeig_batch_query(const ddeig_batch* B, int* ksplit, int* order, int* ntiles,
                               double* tune_us) {
  if (!B) return set_error(DDEIG_EINVAL, "batch is NULL");
  if (ksplit) *ksplit = B->ksplit;
  if (order) *order = B->order;
  if (ntiles) *ntiles = B->ntiles;
  if (tune_us)
    for (int i = 0; i < 6; ++i) tune_us[i] = B->tune_us[i];
  return DDEIG_OK;
}

ddeig_status ddeig_batch_tuning(const ddeig_batch* B, int* tile_rows, double* tune_us) {
  if (!B) return set_error(DDEIG_EINVAL, "batch is NULL");
  if (tile_rows) *tile_rows = B->tile_rows;
  if (tune_us)
    for (int i = 0; i < 12; ++i) tune_us[i] = B->tune_us[i];
  return DDEIG_OK;
}

ddeig_status ddeig_batch_pcg_solve(ddeig_batch* B, const double* const* b, double* const* x,
                                   double rtol, int maxit, ddeig_pcg_info* info) {
  if (!B) return set_error(DDEIG_EINVAL, "batch is NULL");
  if (!b || !x) return set_error(DDEIG_EINVAL, "b or x is NULL");
  if (!(rtol >= 0.0) || !std::isfinite(rtol) || maxit < 0)
    return set_error(DDEIG_EINVAL, "need rtol >= 0 and maxit >= 0");
  for (int j = 0; j < B->n; ++j) {
    if (validate_vec(b[j], "b") || validate_vec(x[j], "x")) return DDEIG_EINVAL;
    if (b[j] == x[j]) return set_error(DDEIG_EINVAL, "b and x must not alias");
    if (!B->P[j]->shifted)
      return set_error(DDEIG_ESTATE, "instance " + std::to_string(j) + ": shift not set");
  }
  API_GUARD_BEGIN
  std::vector<int> active(B->n, 1);
  std::vector<const double*> bb(b, b + B->n);
  std::vector<double*> xx(x, x + B->n);
  batch_pcg(B, active, bb, xx, rtol, maxit);
  ddeig_status st = DDEIG_OK;
  for (int j = B->n - 1; j >= 0; --j) {
    const ddeig::PcgState& h = B->hStates[j];
    if (info) {
      info[j].iters = h.iters;
      info[j].relres = h.relres;
      info[j].breakdown = h.done == 2 ? 1 : (h.done == 3 ? 2 : 0);
      info[j].fallback = 0;
      info[j].true_relres = ddeig::true_relres(B->P[j], b[j], x[j]);
    }
    if (h.done == 2 || h.done == 3)
      st = set_error(DDEIG_ENOTSPD, "instance " + std::to_string(j) + ": CG breakdown");
    else if (h.done != 1 && st != DDEIG_ENOTSPD)
      st = set_error(DDEIG_ENOCONV, "instance " + std::to_string(j) + ": PCG reached maxit");
  }
  return st;
  API_GUARD_END
}

ddeig_status ddeig_batch_inverse_iteration(ddeig_batch* B, double* const* x, double tol_x,
                                           int maxit_outer, double rtol_inner, int maxit_inner,
                                           ddeig_eig_info* info) {
  if (!B) return set_error(DDEIG_EINVAL, "batch is NULL");
  if (!x) return set_error(DDEIG_EINVAL, "x is NULL");
  if (!(tol_x >= 0.0) || maxit_outer < 1 || !(rtol_inner >= 0.0) || maxit_inner < 1)
    return set_error(DDEIG_EINVAL, "invalid tolerances or iteration limits");
  for (int j = 0; j < B->n; ++j) {
    if (validate_vec(x[j], "x")) return DDEIG_EINVAL;
    if (!B->P[j]->shifted)
      return set_error(DDEIG_ESTATE, "instance " + std::to_string(j) + ": shift not set");
  }
  API_GUARD_BEGIN
  const hipStream_t s = B->stream;
  const int n = B->n;
  const auto t0 = std::chrono::steady_clock::now();
  // start vectors: x_j, or 1/||1||_M where x_j is all zeros
  for (int j = 0; j < n; ++j) {
    ddeig_problem* P = B->P[j];
    Red s3 = slot(P, 3);
    launch_dot(x[j], x[j], P->g.n, s3, s);
    if (host_sum(P, s3) == 0.0) {
      launch_fill(P->u, P->g.n, 1.0, s);
      launch_stencil(P, P->tabM, P->u, P->w, &s3, nullptr, s);
      launch_scale_copy(P->g.n, x[j], P->u, s3, s);
    }
  }
  std::vector<int> active(n, 1), status(n, 0), its(n, 0), inner_max(n, 0), unconv(n, 0);
  std::vector<long> inner_sum(n, 0);
  std::vector<double> lam(n, 0.0), dx(n, INFINITY), res(2 * (size_t)n);
  std::vector<const double*> bb(n);
  std::vector<double*> uu(n);
  for (int j = 0; j < n; ++j) {
    bb[j] = B->P[j]->w;
    uu[j] = B->P[j]->u;
    B->inst[j].xo = x[j];
  }
  // every outer step is a fixed set of grouped launches over the active
  // instances: b = M x, the PCG start and iterations, M u, the normalisation,
  // A_sigma x and the two sums per instance
  int* const act_start = B->dAct;
  int* const act_norm = B->dAct + n;
  for (int k = 1; k <= maxit_outer; ++k) {
    int nact = 0;
    for (int j = 0; j < n; ++j) {
      B->hAct[j] = active[j];
      nact += active[j] ? 1 : 0;
    }
    if (nact == 0) break;
    check_hip(hipMemcpyAsync(act_start, B->hAct, sizeof(int) * n, hipMemcpyHostToDevice, s),
              "copy activity");
    batch_upload_inst(B);
    launch_b_stencil_plain(B->dInst, B->bm_st, act_start, 0, s);  // b = M x
    batch_pcg(B, active, bb, uu, rtol_inner, maxit_inner, act_start);
    int nnorm = 0;
    for (int j = 0; j < n; ++j) {
      B->hAct[n + j] = 0;
      if (!active[j]) continue;
      const ddeig::PcgState& h = B->hStates[j];
      if (h.done == 2 || h.done == 3) {
        status[j] = DDEIG_ENOTSPD;
        active[j] = 0;
        continue;
      }
      inner_sum[j] += h.iters;
      inner_max[j] = std::max(inner_max[j], h.iters);
      if (h.done != 1) ++unconv[j];
      its[j] = k;
      B->hAct[n + j] = 1;
      ++nnorm;
    }
    if (nnorm == 0) break;
    check_hip(hipMemcpyAsync(act_norm, B->hAct + n, sizeof(int) * n, hipMemcpyHostToDevice, s),
              "copy activity");
    launch_b_stencil_plain(B->dInst, B->bm_st, act_norm, 1, s);   // M u
    launch_b_normalise(B->dInst, B->bm_node, act_norm, s);         // x = scale u
    launch_b_stencil_plain(B->dInst, B->bm_st, act_norm, 2, s);   // A_sigma x
    launch_b_finish_norm(B->dInst, n, act_norm, B->dRes, s);
    check_launch("batch normalisation");
    check_hip(hipMemcpyAsync(res.data(), B->dRes, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s),
              "copy results");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int j = 0; j < n; ++j) {
      if (!active[j]) continue;
      dx[j] = std::sqrt(std::max(res[2 * j], 0.0));
      lam[j] = B->P[j]->sigma + res[2 * j + 1];
      if (dx[j] <= tol_x) {
        active[j] = 0;
        status[j] = 1;
      }
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  ddeig_status st = DDEIG_OK;
  for (int j = n - 1; j >= 0; --j) {
    if (info) {
      info[j].lambda = lam[j];
      info[j].dx_M = dx[j];
      info[j].outer_its = its[j];
      info[j].inner_sum = inner_sum[j];
      info[j].inner_max = inner_max[j];
      info[j].t_solve_ms = ms;
      info[j].spec_res = ddeig::spectral_residual(B->P[j], x[j], lam[j]);
      info[j].t_setup_ms = B->P[j]->t_setup_ms;
      info[j].inner_unconverged = unconv[j];
      info[j].fallback = 0;
    }
    if (status[j] == DDEIG_ENOTSPD)
      st = set_error(DDEIG_ENOTSPD, "instance " + std::to_string(j) + ": CG breakdown");
    else if (status[j] != 1 && st != DDEIG_ENOTSPD)
      st = set_error(DDEIG_ENOCONV, "instance " + std::to_string(j) + ": reached maxit_outer");
    else if (unconv[j] > 0 && st != DDEIG_ENOTSPD)
      st = set_error(DDEIG_ENOCONV, "instance " + std::to_string(j) +
                                        ": an inner solve stopped at maxit_inner");
  }
  return st;
  API_GUARD_END
}

ddeig_status ddeig_batch_eig_grad(ddeig_batch* B, const double* const* x, double* grad,
                                  int ngrad) {
  if (!B) return set_error(DDEIG_EINVAL, "batch is NULL");
  if (!x || !grad) return set_error(DDEIG_EINVAL, "x or grad is NULL");
  int T = 0;
  for (int j = 0; j < B->n; ++j) {
    if (validate_vec(x[j], "x")) return DDEIG_EINVAL;
    if (grad_params(B->P[j], ngrad, T) != DDEIG_OK) return DDEIG_EINVAL;
  }
  API_GUARD_BEGIN
  std::vector<GradJob> jobs;
  for (int j = 0; j < B->n; ++j) jobs.push_back(grad_job(B->P[j], x[j], x[j], 0));
  std::vector<double> f;
  grad_run(B->allocs, B->gb, jobs, T, B->stream, f);
  const int nf = 2 * T + 1;
  for (int j = 0; j < B->n; ++j) {
    const double* fj = f.data() + (size_t)j * nf;
    if (!(fj[2 * T] > 0.0))
      return set_error(DDEIG_EINVAL, "instance " + std::to_string(j) + ": x^T M x is not positive");
    for (int t = 0; t < 2 * T; ++t) grad[(size_t)j * 2 * T + t] = fj[t] / fj[2 * T];
  }
  return DDEIG_OK;
  API_GUARD_END
}

ddeig_status ddeig_batch_solve_grad(ddeig_batch* B, const double* const* u, const double* const* w,
                                    double* grad, int ngrad) {
  if (!B) return set_error(DDEIG_EINVAL, "batch is NULL");
  if (!u || !w || !grad) return set_error(DDEIG_EINVAL, "u, w or grad is NULL");
  int T = 0;
  for (int j = 0; j < B->n; ++j) {
    if (validate_vec(u[j], "u") || validate_vec(w[j], "w")) return DDEIG_EINVAL;
    if (grad_params(B->P[j], ngrad, T) != DDEIG_OK) return DDEIG_EINVAL;
    if (!B->P[j]->shifted)
      return set_error(DDEIG_ESTATE, "instance " + std::to_string(j) + ": shift not set");
  }
  API_GUARD_BEGIN
  std::vector<GradJob> jobs;
  for (int j = 0; j < B->n; ++j) jobs.push_back(grad_job(B->P[j], B->P[j]->psi, B->P[j]->psi, 1));
  for (int j = 0; j < B->n; ++j) jobs.push_back(grad_job(B->P[j], w[j], u[j], 0));
  std::vector<double> f;
  grad_run(B->allocs, B->gb, jobs, T, B->stream, f);
  const int nf = 2 * T + 1;
  for (int j = 0; j < B->n; ++j) {
    const double* cj = f.data() + (size_t)j * nf;
    const double* gj = f.data() + (size_t)(B->n + j) * nf;
    if (!(cj[2 * T] > 0.0))
      return set_error(DDEIG_ESTATE, "instance " + std::to_string(j) + ": no cell eigenvector");
    for (int t = 0; t < 2 * T; ++t)
      grad[(size_t)j * 2 * T + t] = -(gj[t] - cj[t] / cj[2 * T] * gj[2 * T]);
  }
  return DDEIG_OK;
  API_GUARD_END
}

void ddeig_batch_destroy(ddeig_batch* B) { batch_free(B); }

}  // extern "C"

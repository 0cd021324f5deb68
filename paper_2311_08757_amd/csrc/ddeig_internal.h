// Internal structures of libddeig: geometry, period-cell operator tables,
// subdomain boxes and the kernels' launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ddeig.h"

namespace ddeig {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kBig = 1024;         // workgroup of the node-parallel restriction / extension
constexpr int kRedBlocks = 512;    // grid of the coarse-setup style reducing kernels
constexpr int kMaxRed = 1024;      // largest grid of a reducing kernel (partial-sum capacity)
constexpr int kRedSlots = 16;

// A global sum: the producing kernel writes one partial per block into part
// (np blocks); every consumer adds the np partials in block order, so all
// consumers see the same bits.  val receives the sum when the host needs it.
struct Red {
  double* part;
  int np;
  double* val;
};
constexpr int kMaxTaps = 27;

// Division by a run-time constant d >= 1 through a multiply-high
// (Granlund-Montgomery): q = (umulhi(n, mul) + n) >> shift, exact for n < 2^31.
struct FastDiv {
  unsigned d, mul, shift;
};

inline FastDiv make_fastdiv(unsigned d) {
  FastDiv f{d, 0u, 0u};
  unsigned s = 0;
  while ((1ull << s) < d) ++s;
  f.shift = s;
  f.mul = (unsigned)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}

// Geometry of Omega_L on the internal 3-D index space (N0, N1, N2), dim 0 = x1.
// p + q = D in {2, 3}; for D = 2 the third dim has N2 = 1.  The stencil of a
// node couples the 3^D neighbours; a tap is t = (d0+1) + 3 (d1+1) + 9 (d2+1).
struct Geo {
  int p, q, D;
  int L, ne;
  int nel[3];     // elements per dim
  int N[3];       // interior unknowns per dim
  int P[3];       // period-cell table extent per dim: ne in x dims, N[a] in y dims
  int isx[3];     // 1 for expanding (x) dims
  int ntaps;      // 3^D
  long n;         // N0 N1 N2
  long tsize;     // P0 P1 P2 (table nodes == cell unknowns)
  double h, ell;
  FastDiv fN0, fN1, fne;
};

// Subdomains covering one grid line along an expanding axis: at most two
// cells (2 delta <= n_e), their 1-based index (0: none), the box-local index
// of the node, and the partition-of-unity factor of this axis.
struct XCover {
  int c[2];
  int u[2];
  double w[2];
};

// Potential description copied to the device (see ddeig_potential).
struct VSpec {
  int kind, nterms, p, q;
  double cy, c0, ell;
  double a[DDEIG_MAX_TERMS], phi[DDEIG_MAX_TERMS];
  int k[DDEIG_MAX_TERMS], m[DDEIG_MAX_TERMS];
  double g[3];
  const double* table;  // QUAD_TABLE: device copy of the quadrature-point values
};

// A box of unknowns: origin o[a] (0-based interior unknown index of the first
// node; the cell problem uses o = -1 in x dims so that node index == cell
// index), extent m[a], periodic flag per dim (cell problem only).  Block
// chains run along the last dim (a fixed y direction): slice size
// b = prod_{a < D-1} m[a], chain length m[D-1].
struct Box {
  int o[3];
  int m[3];
  int per[3];
  int b;      // slice size
  int nch;    // chain length
};

// A class of subdomains sharing one local matrix (same cell-local offsets and extents).
struct SubType {
  Box box;                  // box of the first member (o of that member)
  int nmem;
  std::vector<int> members; // subdomain ids (x1-fastest cell numbering)
  double* W = nullptr;      // nch * b * b FP64 Schur-complement inverses
  float* W32 = nullptr;     // FP32 copy (local_prec = 1)
  double* batch = nullptr;  // nmem * nch * b local vectors
  double* phi = nullptr;    // coarse weights of the class (box order)
  // dense local solves (local_prec >= 2): the class box is the node range
  // [off, off + m) of the unclipped box along every axis
  int off[3] = {0, 0, 0};
};

// Dense local solves: the unclipped, period-aligned subdomain box (the box of
// an interior cell), its FP64 block-chain factors, its inverse as bf16 (hi /
// lo) and the batch of all subdomains' restricted residuals R (row = the
// subdomain id, zero outside the subdomain's own box) with the split-K partial
// products Z[split][row][e].
struct DenseHost {
  Box box;
  int m = 0, ld = 0, mp = 0;
  double* W = nullptr;
  __bf16 *Ah = nullptr, *Al = nullptr, *Rh = nullptr, *Rl = nullptr;
  float* Z = nullptr;
};

// A clipped class (a box smaller than the unclipped one): S = its nodes, T =
// the other nodes of the unclipped box, G = B_ST (B_TT)^{-1} for the rounded
// unclipped inverse B, stored t-major over the unclipped box (G[t * mH + e],
// zero for e in T; see k_dense.hip).
struct PcgState;
struct EmbedDev {
  int nT, nmem;
  int off[3], m[3];
  const int* rows;  // batch rows (subdomain ids) of the members
  const int* Tidx;
  const float* G;
  float* Z;         // the problem's split-K products Z[split][row][e]
  long zsplit;
  const PcgState* st;  // CG state checked by grouped launches (nullptr: the launch's own)
  // 1 when the box is clipped along axis 0 only: T is then the columns u0
  // outside [off[0], off[0] + m[0]) of every line, in natural order, and
  // Tidx[t] = u0 + hm0 * line follows from t without a table look-up
  int xonly;
};
// Batch operands of the dense-mode restriction / extension kernels.
struct DenseArgs {
  __bf16* Rh;
  __bf16* Rl;
  const float* Z;
  long zsplit;
  int ld, ksplit, hm0, hm1;
};
struct EmbedJob {
  int cls, mem0, nm;
};
constexpr int kEmbChunk = 8;    // most members per correction block
constexpr int kEmbMaxT = 1024;  // largest T
constexpr int kEmbUT = 8192;    // u_T values per correction block (members x T)
constexpr int kEmbMaxJobs = 65535;  // correction jobs per launch (grid y)
// Members per correction job of a class with nT missing nodes: as many as the
// block's u_T buffer holds (8 at the largest T), at most kEmbChunk.
inline int emb_members_per_job(int nT) {
  const int fit = nT > 0 ? kEmbUT / nT : kEmbChunk;
  return fit < kEmbChunk ? fit : kEmbChunk;
}

// Per-subdomain data on the device.
struct SubDev {
  int o[3];     // box origin
  int type;     // SubType index
  int slot;     // member slot within the type
  int c[3];     // 1-based cell multi-index (x dims), 0 for y dims
};

struct TypeDev {
  int m[3];
  int o[3];           // box origin of the first member (table positions of the class)
  int hm[3], off[3];  // dense batch rows: e = sum_a (u_a + off_a) prod_{b<a} hm_b
  int b, nch;
  const double* W;
  const float* W32;
  double* batch;
  double* tbatch;     // forward-sweep results of the batched chain solves
  // dense local solves (local_prec >= 2): rows of the dense batch (bf16
  // residual, lo part for local_prec = 2) and split-K partial results
  // Z[split][row][e]
  int dense, ld, ksplit;
  __bf16* Rh;
  __bf16* Rl;
  const float* Z;
  long zsplit;
  // coarse weights of the class: phi[e] = D(e) psi_ext(e) on the box of any
  // member (equal for all members by periodicity), and division by m[0]
  const double* phi;
  FastDiv fm0;
  // row stride of the FP32 factors W32 (b, or b rounded up to a multiple of 4
  // for the MFMA chain solves, whose rows are zero padded)
  int ldw;
};

constexpr int kMaxTypes = 9;  // 3 classes per expanding axis, p <= 2

// Subdomain -> (class, slot), packed for the node-parallel kernels.
struct SubTS {
  int type, slot;
};

// Operands of the grouped MFMA GEMM of one dense class (ld x ld inverse).
struct GemmType {
  const __bf16* Ah;
  const __bf16* Al;
  const __bf16* Rh;
  const __bf16* Rl;
  float* Z;
  long zsplit;
  int ld;
  int rows;            // rows of R that hold subdomains (read by the batch's kernels only)
  const PcgState* st;  // CG state checked by grouped launches (nullptr: the launch's own)
};
static_assert(sizeof(GemmType) == 64, "rows sits in the padding after ld");

// Batched chain solves: one workgroup per (class, member tile, 64 rows of a slice).
// Extra workgroups of the dense GEMM launch that form the coarse right-hand
// side R_0 r (one per subdomain), and of the clipped-class correction launch
// that apply the coarse inverse y0 = A_0^{-1} c (four rows per workgroup).
struct CoarseRhsArgs {
  int n;  // subdomains (0: none)
  Geo g;
  const double* r;
  const TypeDev* types;
  const SubDev* subs;
  double* crhs;
};

struct CoarseSolveArgs {
  int n;  // coarse dimension (0: none)
  const double* A0inv;
  const double* c;
  double* y;
};

// A group of at most 64 members of one class in the batched chain solves:
// class, first member within the class, count, and the group's first member
// in the partial-product buffer (members of all classes numbered in order).
struct ChainJob {
  int type, m0, nm, mg0;
};

struct GemmTile {
  int type, m0, n0, k0, k1, split;
};

// Rows [r0, r1) of one small dense class for the streaming kernel.
constexpr int kGemvMax = 4;
struct GemvRows {
  int type, r0, r1, nmem;
};

// PCG device state (one per problem).
struct PcgState {
  int done;      // 0 running, 1 converged, 2 p.Ap <= 0 (CG) / divergence (stationary RAS) /
                 // zero Hessenberg column (GMRES), 3 r.z <= 0, 4 maxit, 5 idle (batch),
                 // 6 end of a GMRES restart cycle
  int iters;
  double rho[2]; // r.z of iterations of even / odd parity
  double r0n2;
  double tol2;
  double relres;
  double rz_floor;  // CG stops with done = 3 when r.z <= rz_floor (0; +inf when a test forces it)
};

// One instance of a batch of problems advanced together: everything the
// grouped kernels of a PCG iteration read, copied to the device once per
// solve.  Each instance keeps its own CG state, scalars and partial sums.
struct InstDev {
  Geo g;
  int delta, pu, nsub;
  int nb_node;  // blocks of the node-parallel restriction / extension
  int nb_cf;    // blocks of the coarse field
  int sty;      // rows of the 2-D stencil tiles (stencil2d_ty)
  int hist_cap;
  const double* tabAs;
  double* x;    // CG iterate
  double *r, *z, *q;
  double* pp[2];
  PcgState* st;
  Red gam, rr, rz;
  DenseArgs da;
  const double* psi;
  double* cf;
  const TypeDev* types;
  const SubDev* subs;
  double* crhs;
  const double* A0inv;
  double* cy;
  const XCover* xc0;
  double* hist;
  // the outer inverse iteration (ddeig_batch_inverse_iteration): mass table,
  // eigenvector iterate, b = M x and the partials of u.Mu, sum(Mu),
  // ||x_new - x||_M^2 and x.A_sigma x
  const double* tabM;
  double* xo;
  double* w;
  Red nm_uMu, nm_sum, nm_dx, nm_xq;
};

// One job of the grouped derivative forms (k_grad.hip): the pair x, y of one
// problem on its grid (cell = 0) or on its periodic cell (cell = 1), the
// problem's potential, its element count, its workgroups and the offset of its
// partial sums (2T + 1 forms x nblk).
struct GradJob {
  Geo g;
  const VSpec* vs;
  const double* x;
  const double* y;
  long nelem;
  int cell, nblk;
  long part0;
};

// Device buffers of the derivative forms, grown on demand.
struct GradBuf {
  GradJob* jobs = nullptr;
  int2* map = nullptr;
  double* part = nullptr;
  double* out = nullptr;
  long cap_jobs = 0, cap_map = 0, cap_part = 0, cap_out = 0;
};

// Block -> (instance, block index within the instance) of a grouped launch.
struct BlockMap {
  const int2* map;
  int nblocks;
};

}  // namespace ddeig

struct ddeig_problem {
  ddeig::Geo g;
  ddeig::VSpec vs;
  int delta;
  ddeig_options opt;
  hipStream_t stream;
  int device = 0;  // the device current at ddeig_assemble
  // second stream (default priority) for work that overlaps the local solves
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // CG state copies of the last two blocks of queued iterations (pinned host
  // memory, so the copies run behind the queued work) and their events
  ddeig::PcgState* hst = nullptr;
  hipEvent_t ev_state[2] = {nullptr, nullptr};
  // HIP-graph replay of PCG iteration blocks (options.graphs): the capture
  // stream and one executable graph per (first, last iteration, maxit, x)
  hipStream_t cap = nullptr;
  std::map<std::tuple<int, int, int, const void*>, hipGraphExec_t> graphs;
  // GMRES step blocks: (cycle start, first step, last step, last step of the
  // cycle, maxit, restart, preconditioner flags, work space)
  std::map<std::tuple<int, int, int, int, int, int, int, const void*>, hipGraphExec_t> gm_graphs;
  // operator tables, tap-major: tab[tap * tsize + tnode]
  double* tabK = nullptr;
  double* tabM = nullptr;
  double* tabA = nullptr;   // K + M_V
  double* tabAs = nullptr;  // A - sigma M
  double* tabW = nullptr;   // M_W of a weight potential W (potential forms)
  ddeig::VSpec* dWS = nullptr;
  double* tmpv = nullptr;   // max(n_dof, n_cell) scratch vector of the potential forms
  ddeig::VSpec* dVS = nullptr;
  // shift
  int shifted = 0;
  double sigma = 0.0;
  double* psi = nullptr;    // tsize cell vector
  // decomposition
  int nsub = 0;
  std::vector<ddeig::SubType> types;
  std::vector<ddeig::SubDev> subs;
  ddeig::SubDev* dSubs = nullptr;
  ddeig::TypeDev* dTypes = nullptr;
  int maxb = 0;
  ddeig::XCover* dXC[2] = {nullptr, nullptr};   // per expanding axis, N[a] entries
  ddeig::SubTS* dSubTS = nullptr;
  int* dFirst = nullptr;          // first member of every class
  double** dPhis = nullptr;       // per-class coarse weights (device pointer array)
  // dense local solves
  ddeig::DenseHost dh;
  std::vector<ddeig::EmbedDev> emb;   // clipped classes (device pointers inside)
  ddeig::EmbedDev* dEmb = nullptr;
  ddeig::EmbedJob* dEmbJobs = nullptr;
  int nembjobs = 0, maxT = 0;
  int ntiles = 0, ngemv = 0, ksplit = 1;
  // batched chain solves (3-D FP64 / FP32 local solves)
  ddeig::ChainJob* dChainJobs = nullptr;
  int nchainjobs = 0;
  int chain_bmax = 0, chain_mtot = 0;  // largest slice, all members of all classes
  void* chain_part = nullptr;          // K-chunk partial products of a sweep step
  int chain_mfma = 0;                  // FP32 chain solves on MFMA (k_chain_mfma.hip)
  ddeig::GemmTile* dTiles = nullptr;
  ddeig::GemvRows* dGemv = nullptr;
  ddeig::GemmType* dGtypes = nullptr;
  // coarse space
  double* A0inv = nullptr;  // nsub x nsub
  double* crhs = nullptr;   // nsub
  double* cy = nullptr;     // nsub
  double* cfield = nullptr; // coarse field sum_c D_c y0_c per expanding-index point (dense solves)
  // work vectors (n each)
  double *r = nullptr, *z = nullptr, *q = nullptr, *u = nullptr, *w = nullptr;
  double* pp[2] = {nullptr, nullptr};  // CG directions of even / odd iterations
  double* red_part = nullptr;   // kRedSlots x kMaxRed partial sums
  double* big_part = nullptr;   // 2 x big_cap partials of kernels with more than kMaxRed workgroups
  long big_cap = 0;
  double* red_val = nullptr;    // kRedSlots results
  ddeig::PcgState* st = nullptr;
  double* hist = nullptr;   // device residual history
  int hist_cap = 0;
  double* scal = nullptr;   // small device scalars
  // SI-preconditioned LOPCG work space (allocated by the first ddeig_lopcg call):
  // 9 vectors, the pointer table of the Gram / update kernels, partial sums
  double* lv = nullptr;
  double** lvp = nullptr;
  double* lpart = nullptr;
  double* lout = nullptr;
  // quadrature-point tables of a QUAD_TABLE potential (device) and of the last
  // QUAD_TABLE weight of potential_form; host copy of the potential's table
  double t_setup_ms = 0.0;  // assemble + shift calls so far (wall time)
  int force_rz = 0;         // PCG solves left that report r.z <= 0 at once (test override)
  int fallbacks = 0;        // switches from dense reduced-precision to FP32 chain local solves
  ddeig::GradBuf gb;        // derivative forms (ddeig_eig_grad and relatives)
  double* dVtab = nullptr;
  double* dWtab = nullptr;
  long wtab_cap = 0;
  std::vector<double> vtab_host;
  // GMRES work space (grown by ddeig_gmres_solve): basis V (gm_cap + 1 vectors),
  // preconditioned basis Z (gm_cap vectors), stride gm_ldv; partials, Hessenberg
  // matrix, rotations and small vectors
  double* gmws = nullptr;
  long gm_ldv = 0;
  int gm_cap = 0;
  int* flag = nullptr;      // factorisation error flag
  double* gjbuf = nullptr;  // Gauss-Jordan row/column buffers (4 x gj_stride)
  int gj_stride = 0;
  double* cellS = nullptr;  // scratch for Schur builds (maxb^2)
  std::vector<void*> allocs;
};

namespace ddeig {

// ---- kernels' host launchers (k_*.hip) ------------------------------------
void launch_build_tables(const ddeig_problem* P, hipStream_t s);
void launch_build_wtable(const ddeig_problem* P, const VSpec* dws, double* tW, hipStream_t s);
long stencil_tiles(const Geo& g);
long stencil_blocks(const ddeig_problem* P);
int stencil2d_ty(const Geo& g);
void launch_shift_table(const ddeig_problem* P, hipStream_t s);
// y = T x (T one of the tables); dot / sum != nullptr: partial sums of x.y / of y
void launch_stencil(const ddeig_problem* P, const double* tab, const double* x, double* y,
                    Red* dot, Red* sum, hipStream_t s);
// PCG iteration k, first kernel: p_k = z + beta_k p_{k-1} (p_1 = z) into pnew,
// q = A_sigma p_k, partials of p_k.q into gam.
struct DirArgs {
  PcgState* st;
  int k;
  Red rz;  // partials of r_{k-1}.z_{k-1}
};
void launch_stencil_dir(const ddeig_problem* P, const double* z, const double* pold, double* pnew,
                        double* q, const DirArgs& dir, Red& gam, hipStream_t s);
void launch_box_stencil(const ddeig_problem* P, const Box& bx, const double* tab, const double* x,
                        double* y, Red* dot, Red* sum, hipStream_t s);

// chain factorisation of a box: W[i] = S_i^{-1}; flag set on a non-positive pivot
void chain_factor(ddeig_problem* P, const Box& bx, const double* tab, double* W, hipStream_t s);
void launch_gj_invert(ddeig_problem* P, double* A, int b, hipStream_t s);
// chain solve in place on nrhs right-hand sides stored contiguously (nch*b each)
void launch_chain_solve_box(const ddeig_problem* P, const Box& bx, const double* tab,
                            const double* W, double* v, int nrhs, hipStream_t s);

// preconditioner pieces
// PCG iteration k, update fused into the restriction: alpha = rho_{k-1} / gamma
// with gamma = p_k.q from the stencil's partials; x += alpha p_k,
// r -= alpha q, partials of ||r||^2 into rr.
struct XrArgs {
  int on, k;
  Red gam;
  double* x;
  const double* p;
  const double* q;
};
// Stopping test of PCG iteration k folded into the extension: the kernel adds
// the ||r_k||^2 partials, records the history and ends CG on convergence or at maxit.
struct CheckArgs {
  int on, k, maxit, hist_cap;
  Red rr;
  double* hist;
};
void launch_restrict(const ddeig_problem* P, double* r, PcgState* st, const XrArgs& xr, Red* rr,
                     hipStream_t s);
void launch_local_solves(const ddeig_problem* P, const PcgState* st, hipStream_t s,
                         const double* coarse_r = nullptr);
bool fused_coarse(const ddeig_problem* P);
int chain_group_members();
size_t chain_part_bytes(int bmax, int mtot, int fp32);
// FP32 batched chain solves on MFMA (k_chain_mfma.hip)
int chain_mfma_members();
bool chain_mfma_ok(int b, int m0);
size_t chain_mfma_part_bytes(int bmax, int mtot);
void launch_chain_mfma(const ddeig_problem* P, const PcgState* st, hipStream_t s);
void launch_pad_float(const double* src, float* dst, long rows, int b, int ldw, hipStream_t s);
void launch_coarse_solve(const ddeig_problem* P, const PcgState* st, hipStream_t s);
void launch_coarse_field(const ddeig_problem* P, const PcgState* st, hipStream_t s);
void launch_coarse_rhs(const ddeig_problem* P, const double* r, const PcgState* st, hipStream_t s);
void launch_coarse_phi(const ddeig_problem* P, hipStream_t s);
void launch_extend(const ddeig_problem* P, const double* r, double* z, int coarse, Red* dot,
                   PcgState* st, const CheckArgs& chk, hipStream_t s, int ras = 0,
                   int inline_field = 0);
void launch_coarse_extend(const ddeig_problem* P, const double* r, double* z, Red* dot,
                          const PcgState* st, hipStream_t s);
void launch_symmetrise(double* A, int N, hipStream_t s);
void launch_split_inverse(const double* Ainv, int m, int ld, void* Ah, void* Al, hipStream_t s);
void launch_identity(double* v, int m, hipStream_t s);
void launch_dense_gemm(const ddeig_problem* P, const PcgState* st, hipStream_t s,
                       const double* coarse_r = nullptr);
void launch_dense_gemv(const ddeig_problem* P, const PcgState* st, hipStream_t s);
void launch_embed_gather(const ddeig_problem* P, const EmbedDev& E, double* C, hipStream_t s);
void launch_embed_gmat(const ddeig_problem* P, const EmbedDev& E, const double* C, float* G,
                       hipStream_t s);
void launch_embed_fix(const ddeig_problem* P, const PcgState* st, hipStream_t s,
                      bool coarse_solve = false);
void launch_to_float(const double* src, float* dst, long n, hipStream_t s);
void build_coarse_matrix(ddeig_problem* P, double* A0, hipStream_t s);

// grouped launches over the instances of a batch (one PCG iteration k)
int node_grid(const Geo& g);
int node_grid_dense(const Geo& g);
int coarse_field_grid(const Geo& g);
void launch_b_stencil_dir(const InstDev* I, const BlockMap& bm, int k, hipStream_t s);
void launch_b_restrict(const InstDev* I, const BlockMap& bm, int k, hipStream_t s);
void launch_b_extend(const InstDev* I, const BlockMap& bm, int k, int maxit, int ksplit,
                     hipStream_t s, int check = 1);
void launch_b_coarse_rhs(const InstDev* I, const BlockMap& bm, hipStream_t s);
void launch_b_coarse_solve(const InstDev* I, const BlockMap& bm, hipStream_t s);
void launch_b_coarse_field(const InstDev* I, const BlockMap& bm, hipStream_t s);
void launch_gemm_tiles(const GemmTile* tiles, int ntiles, const GemmType* gt, int local_prec,
                       hipStream_t s, int tile_rows = 128);
void launch_embed_jobs(const EmbedJob* jobs, int njobs, const EmbedDev* cls, int ksplit, int ld,
                       int hm0, int hm1, int mH, hipStream_t s);
void launch_b_states(const InstDev* I, int n, PcgState* out, int mark_done, hipStream_t s);
void launch_b_restrict_start(const InstDev* I, const BlockMap& bm, const int* act, hipStream_t s);
void launch_b_pcg_init(const InstDev* I, int n, const int* act, double rtol, hipStream_t s);
void launch_b_normalise(const InstDev* I, const BlockMap& bm, const int* act, hipStream_t s);
void launch_b_finish_norm(const InstDev* I, int n, const int* act, double* res, hipStream_t s);
void launch_b_stencil_plain(const InstDev* I, const BlockMap& bm, const int* act, int which,
                            hipStream_t s);

// PCG / IPM vector kernels
int red_grid(long work_items);
void launch_resid_init(const ddeig_problem* P, const double* b, const double* q, double* r,
                       Red& rr, hipStream_t s);
void launch_finish_sum(const Red& r, hipStream_t s);
void launch_pcg_init(const ddeig_problem* P, double rtol, Red rr, hipStream_t s,
                     double rz_floor = 0.0);
void launch_fill(double* x, long n, double v, hipStream_t s);
void launch_copy(double* dst, const double* src, long n, hipStream_t s);
void launch_scale_copy(long n, double* dst, const double* src, Red nrm2, hipStream_t s);
void launch_ipm_normalise(long n, const double* u, const double* Mu, double* x, const double* b,
                          Red uMu, Red sumMu, Red& dx, hipStream_t s);
void launch_dot(const double* x, const double* y, long n, Red& out, hipStream_t s);

// SI-preconditioned LOPCG (k_vector.hip); dv: device array of vector pointers
constexpr int kLopcgQ = 15;  // Gram quantities of one outer step
void launch_lopcg_orth(long n, double alpha, double beta, const double* x, double* w, double* xp,
                       hipStream_t s);
// dv = {x, w, p, Ax, Aw, Ap, Bx, Bw, Bp}; out[0..14] (see k_lopcg_gram)
int launch_lopcg_gram(long n, const double* const* dv, double* part, double* out, hipStream_t s);
void launch_lopcg_update(long n, double c0, double c1, double c2, double* x, const double* w,
                         double* p, hipStream_t s);
int launch_lopcg_resid(long n, double lambda, const double* Ax, const double* Bx, double* r,
                       double* part, double* out, hipStream_t s);

// Stationary RAS and GMRES (k_krylov.hip)
void launch_sr_update(const ddeig_problem* P, const double* z, double* x, hipStream_t s);
void launch_sr_check(const ddeig_problem* P, const Red& rr, int k, int maxit, hipStream_t s);
int gm_blocks(long n);
long gm_stride(long n);
constexpr int kGmMaxRestart = 1024;  // largest GMRES restart length (LDS of k_gm_decide)
void launch_gm_dots(const ddeig_problem* P, int j, const double* V, long ldv, const double* w,
                    double* part, hipStream_t s);
void launch_gm_sum(const ddeig_problem* P, int rows, const double* part, double* out,
                   hipStream_t s);
void launch_gm_decide(const ddeig_problem* P, int j, int k, int maxit, int restart, int has_w,
                      const double* d, double* H, double* cs, double* sn, double* g, double* cv,
                      double* gm, hipStream_t s);
void launch_gm_update_basis(const ddeig_problem* P, int j, double* V, long ldv, const double* w,
                            const double* d, const double* gm, hipStream_t s);
void launch_gm_start(const ddeig_problem* P, const Red& rr, const double* r, double* v0, double* g,
                     double* gm, hipStream_t s);
void launch_gm_update(const ddeig_problem* P, int nv, const double* Z, long ldv, const double* y,
                      double* x, hipStream_t s);

void check_hip(hipError_t e, const char* what);

// Derivative forms (k_grad.hip): grouped launch over jobs, T Fourier terms.
int grad_blocks(long nelem);
void launch_grad_forms(const GradJob* dJobs, const int2* dMap, int nblocks, int njobs, int T,
                       double* part, double* out, hipStream_t s);

// The potential form without device allocation (k_noalloc.hip).
hipError_t noalloc_init(int dev);
ddeig_status noalloc_form_checked(ddeig_problem* P, int space, const VSpec& wspec, const double* table,
                                  long table_len, const double* x, const double* y, double* out,
                                  std::string& err);

}  // namespace ddeig

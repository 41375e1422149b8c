// C-ABI and orchestration of the SG wave solver on one MI355X.
//
// One time step (Alg. 1 loop body, SG form of Sec. 5):
//   H1  Newmark predictor and effective force F~ = (I(x)M) Um + C Uc
//   H2  static condensation: Dirichlet solves per subdomain, G = F_G - K_GI x_I
//   H3  interface initial guess
//   H4  PCG on S U_G = G with the two-level Neumann-Neumann preconditioner
//   H5  interior recovery, accumulated from the Schur applies of H4 (no
//       Dirichlet solve of its own)
//   H6  Newmark update
// The subdomain solves with the SG-coupled matrices (H8) run as batched
// block-PCG with the mean-matrix preconditioner I_P (x) (K~_0^s)^{-1}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "coarse.h"
#include "kernels.h"
#include "mlp.h"
#include "setup.h"
#include "sgw.h"

using namespace sgw;

// Refinement path (SGW_FP32_IR64): tolerances of each FP32 DD solve and the
// sweep cap of the FP64 refinement loop.
static const double kIrOuterRtol = 1e-5;    // interface PCG, relative to ||G||
static const double kIrInnerRtol = 1e-6;    // Dirichlet solves (the operator)
static const double kIrPrecondRtol = 1e-3;  // Neumann solves (the preconditioner)
static const int kIrMaxSweeps = 8;

namespace {

template <typename T>
struct SysT {  // batched block-diagonal SG system (Dirichlet or Neumann)
  int nrows = 0, nb = 0, Q = 8;
  int cq = 8, max_block_rows = 0;     // Chebyshev mode tile, largest block
  int cshape = 0;                     // Chebyshev launch shape (k::cheb_apply)
  const k::DHalo* halo = nullptr;     // 64-row group halos of A (both precisions)
  const T* cheb_cc = nullptr;         // device, [nb][2 deg] Chebyshev step coefficients
  const int* lpt = nullptr;           // device, blocks by decreasing size (launch order)
  const int* crow = nullptr;          // device, system row of each natural block position
  const unsigned short* cnb = nullptr;  // device, [nrows][8] neighbours' natural positions
  const T* cval = nullptr;            // device, [nrows][8] mean-matrix rows, natural order
  // iteration count of the previous solve, by call site (see inner_solve)
  // and tolerance class (tight / loose)
  int last_its[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double loose_tol = 1e300;     // tolerances >= this use the second count
  k::DEll<T> A;
  k::DFactor F;
  const int* row_off = nullptr;  // device
  T *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  T* p2 = nullptr;  // second direction buffer of the fused iteration (alternates with p)
};

// Everything one precision of the DD solve needs: the global operator, the
// Dirichlet and Neumann systems, the interface PCG vectors (full [P][NF]
// arrays, interface part at offset nI) and the torn Neumann buffers.
template <typename T>
struct PrecT {
  bool ready = false;
  k::DEll<T> G;
  SysT<T> D, N;
  T *X = nullptr, *R = nullptr, *Z = nullptr, *Zp = nullptr, *Pw = nullptr, *Qw = nullptr,
    *T1 = nullptr, *Gv = nullptr, *Tt = nullptr, *Yt = nullptr;
  T *Fb = nullptr, *Xb = nullptr;  // right-hand side and correction of a refinement sweep
};

// tolerances of one DD solve
struct Tols {
  double rtol, inner, precond;
  int max_iter, inner_max_iter;
};

}  // namespace

struct sgw_ctx {
  Host h;
  sgw_allocator al{};
  bool has_al = false;
  std::vector<void*> mem;
  std::string err;
  int dev = 0;
  int P = 0, nk = 0, NF = 0, nI = 0, nG = 0, nC = 0, NT = 0, nsub = 0, nn = 0;
  k::GTab gt;
  PrecT<double> d64;
  PrecT<float> f32;
  k::DCoarse co;
  k::DCoarseFactor cf;  // block-bidiagonal factor of F_cc (sgw_factor)
  double *U = nullptr, *V = nullptr, *A = nullptr, *Um = nullptr, *Uc = nullptr,
         *Wm = nullptr, *F = nullptr, *meshbuf = nullptr, *meshbuf2 = nullptr;
  // K~ U, K~ V, K~ A (refinement path with stiffness damping): the damping
  // share of the force follows from them without an SG apply; g_valid once
  // they belong to the current state
  double *GU = nullptr, *GV = nullptr, *GA = nullptr;
  bool g_valid = false;
  double *part = nullptr, *part2 = nullptr, *sc = nullptr, *dc = nullptr, *uc = nullptr;
  double* osc = nullptr;   // interface PCG: G'G and r'r partials, device scalars
  double* hosc = nullptr;  // pinned copy of osc
  int* flags = nullptr;
  int* hflags = nullptr;
  std::vector<int> crow_h[2];  // natural order of the Dirichlet / Neumann blocks (host)
  const int* goff = nullptr;   // row chunks of [0, nG), relative to an interface-part pointer
  int ngchunk = 1;
  const int* alloff = nullptr; // {0, NF}
  const int* fchunk = nullptr;  // row chunks of [0, NF) for the whole-array dot products
  int nfchunk = 0;
  double* hpart = nullptr;      // pinned, 2 x nfchunk x P partial sums
  const int* dd2mesh = nullptr;
  const double* mdiag = nullptr;
  // interface <-> torn maps
  const int *torn_gidx = nullptr, *gam_ptr = nullptr, *gam_torn = nullptr, *g2c = nullptr;
  const double *torn_w = nullptr, *gam_w = nullptr;
  int maxc = 0;
  std::vector<int> rem_off_h, rem_list_h;
  std::vector<long long> phi_off_h, phih_off_h;
  double* phi = nullptr;
  unsigned short* phih = nullptr;  // FP16 copy of phi (FP32 solver)
  double* fs = nullptr;   // local coarse matrices during factor
  bool factored = false, has_state = false;
  long long stepno = 0;
  // kernel timing: event pairs around SG-apply (kind 0), triangular-solve
  // (kind 1) and Chebyshev (kind 2) launches in FP64 (kinds 3-5: the same in
  // FP32), every prof_every-th launch of a kind; launches, milliseconds and
  // algorithmic bytes per kind
  bool prof = false;
  int prof_every = 1;
  unsigned long long* acct = nullptr;   // device [4]: bytes of timed K3c FP64 / FP32 and
                                        // fused SG-apply FP64 / FP32 launches (counted by them)
  unsigned long long* acct_h = nullptr; // pinned copy
  bool acct_staged = false;             // acct_h holds the counters (prof_stage)
  unsigned long long acct_seen[4] = {0, 0, 0, 0};
  long long pseen[6] = {0, 0, 0, 0, 0, 0};
  std::vector<hipEvent_t> ev;
  struct Pend { int a, kind; double bytes; };
  std::vector<Pend> pend;
  long long pcnt[6] = {0, 0, 0, 0, 0, 0};
  double pms[6] = {0, 0, 0, 0, 0, 0}, pbytes[6] = {0, 0, 0, 0, 0, 0};
  // 64-row group halos of the SG-apply matrices: global system from row 0
  // and from the first interface row, Dirichlet and Neumann systems
  k::DHalo hal_G0, hal_GI, hal_D, hal_N;
  int k1_generated[2] = {0, 0};  // generated SG-apply kernels (output groups), FP32 / FP64
  double* pqg = nullptr;       // [groups][P] p'q partials of the fused SG apply
  // learned initial guess: ring of the last 4 converged interface solutions
  // [4][P][nG], the Newmark guess of the current step [P][nG], per-mode
  // scales [P], network input/output [P][4 nG] / [P][nG], the attached
  // model and the sample recorder (caller's device arrays)
  double *hist = nullptr, *gnew = nullptr, *smax = nullptr;
  int hist_n = 0, hist_pos = 0;
  float *mx = nullptr, *my = nullptr;
  sgw_mlp* mlp = nullptr;
  hipStream_t own_stream = nullptr;  // created by sgw_step_batch when no stream is given
  // captured pairs of inner PCG iterations (desc.graphs): key = system,
  // tolerance; captured on cap_stream, replayed on the solve's stream
  bool use_graphs = false;
  hipStream_t cap_stream = nullptr;
  struct GraphKey {
    const void* sys;
    double tol2;
    bool operator<(const GraphKey& o) const {
      return sys != o.sys ? sys < o.sys : tol2 < o.tol2;
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  long long graph_launches = 0;
  float *rec_x = nullptr, *rec_t = nullptr;
  long long rec_cap = 0, rec_n = 0;
  // sample store of sgw_guess_train: [cap][4] inputs, [cap] targets
  float *gs_x = nullptr, *gs_t = nullptr;
  long long gs_cap = 0, gs_n = 0;
  long long guess_fallbacks = 0;  // learned guesses replaced by the Newmark guess
  // subdomain preconditioner: SGW_INNER_* and the Chebyshev degree
  int inner_prec = SGW_INNER_CHOLESKY, cheb_deg = 4;
  double factor_bytes_D = 0, factor_bytes_N = 0;
  // per-call statistics
  long long inner_its = 0;
  int inner_solves = 0;
  int status_warn = 0;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
#define HIPCHK(x)                                                         \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      c->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " \
               + #x;                                                      \
      return SGW_EHIP;                                                    \
    }                                                                     \
  } while (0)

static void* dalloc_bytes(sgw_ctx* c, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  void* p = nullptr;
  if (c->has_al) {
    p = c->al.alloc(bytes, c->al.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    c->mem.push_back(p);
    (void)hipMemset(p, 0, bytes);  // no kernel ever sees uninitialised memory
  }
  return p;
}

// Releases one allocation of dalloc_bytes before sgw_destroy.
static void dfree(sgw_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->mem.begin(), c->mem.end(), p);
  if (it == c->mem.end()) return;
  c->mem.erase(it);
  if (c->has_al) c->al.free(p, c->al.user);
  else (void)hipFree(p);
}

template <class T>
static T* dalloc(sgw_ctx* c, size_t n) {
  return reinterpret_cast<T*>(dalloc_bytes(c, n * sizeof(T)));
}

template <class T>
static T* upload(sgw_ctx* c, const std::vector<T>& v) {
  T* d = dalloc<T>(c, v.size());
  if (d && !v.empty() &&
      hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return nullptr;  // reported by the completeness check of sgw_create
  return d;
}

static std::vector<float> to_f(const std::vector<double>& v) {
  return std::vector<float>(v.begin(), v.end());
}

// Galerkin contraction table for the SG apply kernel (see kernels.h).
static int build_gtab(sgw_ctx* c, int KC, int GS) {
  const Galerkin& g = c->h.g;
  k::GTab t;
  t.nk = g.nk;
  t.P = g.P;
  t.KC = KC;
  t.GS = GS;
  t.ng = (g.P + GS - 1) / GS;
  t.nch = (g.nk + KC - 1) / KC;
  t.L = g.L;
  t.p_in = g.p_in;
  t.p_out = g.p_out;
  const char* env = getenv("SGW_K1_GENERIC");
  t.use_spec = !(env && env[0] == '1');
  std::map<std::pair<int, int>, std::vector<std::pair<int, double>>> byKJ;
  for (size_t e = 0; e < g.v.size(); ++e) byKJ[{g.k[e], g.j[e]}].push_back({g.i[e], g.v[e]});
  std::vector<uint32_t> mask;
  std::vector<int> pbeg, ebeg, pcnt, ei;
  std::vector<double> ec;
  for (int grp = 0; grp < t.ng; ++grp)
    for (int ch = 0; ch < t.nch; ++ch)
      for (int j = 0; j < g.P; ++j) {
        uint32_t m = 0;
        pbeg.push_back((int)pcnt.size());
        ebeg.push_back((int)ei.size());
        for (int kk = 0; kk < KC; ++kk) {
          int kx = ch * KC + kk;
          if (kx >= g.nk) break;
          auto it = byKJ.find({kx, j});
          if (it == byKJ.end()) continue;
          int cnt = 0;
          for (auto& iv : it->second)
            if (iv.first >= grp * GS && iv.first < (grp + 1) * GS) {
              ei.push_back(iv.first - grp * GS);
              ec.push_back(iv.second);
              ++cnt;
            }
          if (cnt) {
            m |= 1u << kk;
            pcnt.push_back(cnt);
          }
        }
        mask.push_back(m);
      }
  t.mask = upload(c, mask);
  t.pair_beg = upload(c, pbeg);
  t.ent_beg = upload(c, ebeg);
  t.pair_cnt = upload(c, pcnt);
  t.ent_i = upload(c, ei);
  t.ent_c = upload(c, ec);
  t.ent_cf = upload(c, to_f(ec));
  c->gt = t;
  return 0;
}

static k::DFactor upload_factor(sgw_ctx* c, const Factor& f) {
  k::DFactor d;
  d.nb = f.nb;
  d.P = c->P;
  d.row_off = upload(c, f.row_off);
  d.lvl_off = upload(c, f.lvl_off);
  d.lvl_ptr = upload(c, f.lvl_ptr);
  d.lrow_ptr = upload(c, f.lrow_ptr);
  d.lrow_list = upload(c, f.lrow_list);
  d.lrow_sn = upload(c, f.lrow_sn);
  d.lvl_gf = upload(c, f.lvl_gf);
  d.lvl_gb = upload(c, f.lvl_gb);
  d.sn_beg = upload(c, f.sn_beg);
  d.sn_w = upload(c, f.sn_w);
  d.sn_dinv = upload(c, f.sn_dinv);
  d.lr_ptr = upload(c, f.lr_ptr);
  d.lr_col = upload(c, f.lr_col);
  d.lc_ptr = upload(c, f.lc_ptr);
  d.lc_row = upload(c, f.lc_row);
  d.lr_val = upload(c, f.lr_val);
  d.lc_val = upload(c, f.lc_val);
  d.dinv = upload(c, f.dinv);
  d.dinvT = upload(c, f.dinvT);
  d.dinvTf = upload(c, to_f(f.dinvT));
  d.lr_valf = upload(c, to_f(f.lr_val));
  d.lc_valf = upload(c, to_f(f.lc_val));
  d.dinvf = upload(c, to_f(f.dinv));
  d.max_rows = f.max_rows;
  d.max_level_rows = f.max_level_rows;
  d.max_sn = f.max_sn;
  d.max_levels = f.max_levels;
  d.max_lvl_d = f.max_lvl_d;
  return d;
}

// ---------------------------------------------------------------------------
// kernel timing (sgw_profile): a HIP event pair around each timed launch,
// harvested at the host synchronisation points the solver has anyway.
// ---------------------------------------------------------------------------
// record = false: the caller's launch records the pair itself
// (hipExtLaunchKernelGGL, with the kernel's dispatch).
static int prof_begin(sgw_ctx* c, int kind, hipStream_t st, bool record = true) {
  if (!c->prof) return -1;
  if (c->pseen[kind]++ % c->prof_every != 0) return -1;
  int a = (int)c->pend.size() * 2;
  while ((int)c->ev.size() < a + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    c->ev.push_back(e);
  }
  if (record) (void)hipEventRecord(c->ev[a], st);
  return a;
}
static void prof_end(sgw_ctx* c, int a, int kind, double bytes, hipStream_t st,
                     bool record = true) {
  if (a < 0) return;
  if (record) (void)hipEventRecord(c->ev[a + 1], st);
  c->pend.push_back({a, kind, bytes});
}
// Before a stream synchronisation: the device byte counters are copied on
// the stream, so the harvest after it needs no copy of its own.
static void prof_stage(sgw_ctx* c, hipStream_t st) {
  if (c->pend.empty() || !c->acct) return;
  c->acct_staged = hipMemcpyAsync(c->acct_h, c->acct, 4 * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, st) == hipSuccess;
}
static void prof_harvest(sgw_ctx* c) {
  if (c->pend.empty()) return;
  const bool staged = c->acct_staged;
  c->acct_staged = false;
  if (c->acct && (staged || hipMemcpy(c->acct_h, c->acct, 4 * sizeof(unsigned long long),
                                      hipMemcpyDeviceToHost) == hipSuccess)) {
    static const int kind_of[4] = {2, 5, 0, 3};
    for (int q = 0; q < 4; ++q) {
      c->pbytes[kind_of[q]] += (double)(c->acct_h[q] - c->acct_seen[q]);
      c->acct_seen[q] = c->acct_h[q];
    }
  }
  for (auto& p : c->pend) {
    float ms = 0.f;
    if (hipEventSynchronize(c->ev[p.a + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, c->ev[p.a], c->ev[p.a + 1]) == hipSuccess) {
      c->pcnt[p.kind] += 1;
      c->pms[p.kind] += ms;
      c->pbytes[p.kind] += p.bytes;
    }
  }
  c->pend.clear();
}

// K1 wrapper: algorithmic bytes per row = 7 (M+1) values + 7 column indices
// + P inputs + P outputs (+ P when the output is accumulated).
template <typename T>
static void K1(sgw_ctx* c, const k::DEll<T>& A, const k::DHalo* H, int r0, int nrows, const T* x,
               int ldx, T* y, int ldy, double alpha, double beta, hipStream_t st) {
  const int kind = sizeof(T) == 4 ? 3 : 0;
  int a = prof_begin(c, kind, st);
  k::sg_apply<T>(A, c->gt, H, r0, nrows, x, ldx, y, ldy, (T)alpha, (T)beta, 1, 0, 0, st);
  const double w = sizeof(T);
  double per_row = 7.0 * c->nk * w + 7.0 * 4.0 + 2.0 * c->P * w + (beta != 0.0 ? c->P * w : 0.0);
  prof_end(c, a, kind, per_row * nrows, st);
}

// K3 wrapper: algorithmic bytes = right-hand sides in and out + the factor.
template <typename T>
static void K3(sgw_ctx* c, SysT<T>& S, bool neumann, const T* rhs, int ldr, T* out, int ldo,
               hipStream_t st) {
  const int kind = sizeof(T) == 4 ? 4 : 1;
  int a = prof_begin(c, kind, st);
  k::tri_solve<T>(S.F, S.Q, rhs, ldr, out, ldo, 1, 0, 0, st);
  double fb = (neumann ? c->factor_bytes_N : c->factor_bytes_D) * (sizeof(T) / 8.0);
  prof_end(c, a, kind, 2.0 * sizeof(T) * c->P * S.nrows + fb, st);
}

// Subdomain preconditioner z = (I_P (x) (K~_0^s)^{-1}) r on the system's
// [P][nrows] vectors r, z, followed by the partial sums part[b*P + j] =
// r_j'z_j (and part2 = r_j'r_j if not null).  Exact (K3 + K4) or Chebyshev
// (K3c, one fused launch; algorithmic bytes: r in, z out, the mean
// matrix's values and column indices).  test_par >= 0 first runs the PCG
// stopping test of that iteration (fused into K3c, which then skips the
// converged blocks).
template <typename T>
static void precond_dot(sgw_ctx* c, SysT<T>& S, bool neumann, double* part, double* part2,
                        int test_par, double tol2, hipStream_t st) {
  const int P = c->P, n = S.nrows;
  if (c->inner_prec == SGW_INNER_CHEBYSHEV) {
    const int kind = sizeof(T) == 4 ? 5 : 2;
    int a = prof_begin(c, kind, st, false);
    // timed launches count their bytes on the device (converged blocks are
    // skipped inside the kernel; harvested into the kind's total) and have
    // their event pair recorded by the launch itself
    (void)k::cheb_apply<T>(S.cval, S.row_off, S.lpt, S.crow, S.cnb, S.cheb_cc, S.nb, P,
                           c->cheb_deg,
                           S.cq, S.cshape, S.max_block_rows, S.r, n, S.z, n, part, part2,
                           test_par >= 0 ? c->sc : nullptr, std::max(test_par, 0), tol2,
                           c->part2, c->flags, a >= 0 ? c->acct + (sizeof(T) == 4) : nullptr, st,
                           a >= 0 ? c->ev[a] : nullptr, a >= 0 ? c->ev[a + 1] : nullptr);
    prof_end(c, a, kind, 0.0, st, false);
    return;
  }
  if (test_par >= 0) k::pcg_test(S.nb, P, test_par, c->part2, c->sc, tol2, c->flags, st);
  K3<T>(c, S, neumann, S.r, n, S.z, n, st);
  k::seg_dot<T>(S.nb, S.row_off, P, S.r, n, S.z, n, part, part2 ? S.r : nullptr, n,
                part2 ? S.r : nullptr, n, part2, st);
}

// ---------------------------------------------------------------------------
// H8: batched subdomain SG solves.  PCG per block with x0 = 0 and the
// preconditioner I_P (x) (K~_0^s)^{-1} (exact or Chebyshev); block b stops
// when ||r_b|| <= tol ||b_b||, converged blocks are frozen (alpha = 0).  Per
// iteration: SG apply (K1), p'q partial sums (K4), x/r update with the step
// lengths computed in place, preconditioner with the stopping test, p update
// with beta computed in place.  The iteration count of the previous solve of
// the same system and tolerance class tells the host when to start reading
// the active count: extra iterations of frozen blocks change nothing.
// ---------------------------------------------------------------------------
// Relative size (squared norms) below which a block's right-hand side is
// negligible within its batch: FP64 solves every nonzero block, FP32 leaves
// blocks 1e-10 below the largest at zero (their values can underflow FP32).
template <typename T> struct NegligibleBlock { static constexpr double value = 0.0; };
template <> struct NegligibleBlock<float> { static constexpr double value = 1e-20; };

// Captures (once per system and tolerance) what enqueue() launches into an
// executable graph.  Capture runs on a private stream and executes nothing.
template <class Enqueue>
static int pair_graph(sgw_ctx* c, const void* sys, double tol2, Enqueue enqueue,
                      hipGraphExec_t* out) {
  const sgw_ctx::GraphKey key{sys, tol2};
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return 0;
  }
  if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->err = "stream creation failed";
    return SGW_EHIP;
  }
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->err = "graph capture could not start";
    return SGW_EHIP;
  }
  enqueue(c->cap_stream);
  if (hipStreamEndCapture(c->cap_stream, &g) != hipSuccess ||
      hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    c->err = "graph capture failed";
    return SGW_EHIP;
  }
  (void)hipGraphDestroy(g);
  c->graphs[key] = ge;
  *out = ge;
  return 0;
}

// Call sites of inner_solve, each with its own iteration prediction.
enum { kSiteSchur = 0, kSiteNeumann = 1, kSiteCondense = 2 };

// Batched block PCG.  The host reads the device's convergence flags only
// once the predicted number of iterations (that of the previous solve from
// the same call site) has been issued, then after every further iteration;
// a block that has converged is frozen (every kernel of an iteration skips
// it), so iterations issued past its convergence cost a few microseconds.
template <typename T>
static int inner_solve(sgw_ctx* c, SysT<T>& S, bool neumann, const T* b, int ldb, T* out,
                       int ldo, double tol, int maxit, int site, hipStream_t st) {
  const int P = c->P, n = S.nrows, nb = S.nb;
  const double tol2 = tol * tol;
  int& predicted = S.last_its[2 * site + (tol >= S.loose_tol ? 1 : 0)];
  // fused iteration: the SG apply also forms p (alternating buffers) and the
  // p'q partial sums (generated kernel on a block-aligned halo)
  const int kgen = c->k1_generated[sizeof(T) == 8];
  const bool fused = kgen > 0 && S.halo && k::sg_apply_pcg_fits<T>(c->gt, *S.halo);
  // the iterate lives in the caller's output, except under graph replay,
  // whose captured launches keep the system's own array
  T* const x = c->use_graphs ? S.x : out;
  const int ldx = c->use_graphs ? n : ldo;
  k::copy2d<T, T>(P, n, b, ldb, S.r, n, 1.0, st);
  k::fill2d<T>(P, n, x, ldx, T(0), st);
  precond_dot<T>(c, S, neumann, c->part, c->part2, -1, 0.0, st);
  if (!fused) k::copy2d<T, T>(P, n, S.z, n, S.p, n, 1.0, st);
  k::pcg_start(nb, P, c->part, c->part2, c->sc, tol2, NegligibleBlock<T>::value, c->flags, st);
  int it = 0, rc = 0;
  int nact = 1;
  int done = 0;  // iterations of the slowest block (device count)
  if (predicted <= 1) {
    HIPCHK(hipMemcpyAsync(c->hflags, c->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    nact = c->hflags[0];
    if (c->hflags[2]) {
      c->err = "non-finite residual in a subdomain solve";
      return SGW_ENAN;
    }
  }
  // one iteration up to the stopping test, and its p update
  auto first_half = [&](int par, hipStream_t s) {
    if (fused) {
      T* pold = par ? S.p : S.p2;
      T* pnew = par ? S.p2 : S.p;
      // timed launches count the algorithmic bytes of the rows they process
      // (row groups of converged blocks exit at once) on the device: those
      // of one SG apply, 7 (M+1) values + 7 column indices + one vector in
      // and one out per row (the fused p update moves two more vectors,
      // reported apart from these)
      const int a = prof_begin(c, sizeof(T) == 4 ? 3 : 0, s);
      const unsigned bpr = (unsigned)(7 * c->nk * sizeof(T) + 7 * 4 + 2 * P * sizeof(T));
      (void)k::sg_apply_pcg<T>(S.A, c->gt, *S.halo, n, pold, S.z, pnew, n, S.q, c->part, c->sc,
                               par, c->pqg, a >= 0 ? c->acct + 2 + (sizeof(T) == 4) : nullptr,
                               bpr, s);
      prof_end(c, a, sizeof(T) == 4 ? 3 : 0, 0.0, s);
      k::pcg_xr<T>(nb, S.row_off, P, par, c->sc, x, ldx, pnew, n, S.r, n, S.q, n, c->pqg,
                   c->part2, c->flags, s, S.halo->bgrp, kgen);
    } else {
      K1<T>(c, S.A, S.halo, 0, n, S.p, n, S.q, n, 1.0, 0.0, s);
      k::seg_dot<T>(nb, S.row_off, P, S.p, n, S.q, n, c->part, nullptr, 0, nullptr, 0, nullptr,
                    s);
      k::pcg_xr<T>(nb, S.row_off, P, par, c->sc, x, ldx, S.p, n, S.r, n, S.q, n, c->part,
                   c->part2, c->flags, s);
    }
    precond_dot<T>(c, S, neumann, c->part, nullptr, par, tol2, s);
  };
  auto second_half = [&](int par, hipStream_t s) {
    if (!fused) k::pcg_p<T>(nb, S.row_off, P, par, c->sc, c->part, S.z, n, S.p, n, s);
  };
  // H9: while no stopping test is due, pairs of iterations (even, odd)
  // replay a captured graph; frozen blocks make extra iterations harmless
  if (c->use_graphs && !c->prof && nact > 0) {
    hipGraphExec_t ge = nullptr;
    while (it + 2 <= predicted && it + 2 <= maxit) {
      if (!ge) {
        int grc = pair_graph(c, &S, tol2, [&](hipStream_t s) {
          first_half(0, s);
          second_half(0, s);
          first_half(1, s);
          second_half(1, s);
        }, &ge);
        if (grc) return grc;
      }
      HIPCHK(hipGraphLaunch(ge, st));
      c->graph_launches++;
      it += 2;
    }
  }
  while (nact > 0) {
    if (it >= maxit) {
      rc = SGW_NOT_CONVERGED;
      break;
    }
    const int par = it & 1;
    first_half(par, st);
    ++it;
    if (it >= predicted || it >= maxit) {
      HIPCHK(hipMemcpyAsync(c->hflags, c->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
      prof_stage(c, st);
      HIPCHK(hipStreamSynchronize(st));
      prof_harvest(c);
      nact = c->hflags[0];
      done = c->hflags[3];
      if (c->hflags[1]) {
        c->err = "breakdown (p'q <= 0) in a subdomain solve";
        return SGW_EBREAKDOWN;
      }
      if (c->hflags[2]) {
        c->err = "non-finite residual in a subdomain solve";
        return SGW_ENAN;
      }
      if (nact == 0) break;
    }
    second_half(par, st);
  }
  if (x != out) k::copy2d<T, T>(P, n, x, n, out, ldo, 1.0, st);
  predicted = done;
  c->inner_its += done;
  c->inner_solves += 1;
  return rc;
}

// q_G = S p_G (Eq. Sto_Schur): harmonic extension of p into the interiors
// (Dirichlet solves) and the interface rows of the global operator.  w and q
// are full [P][NF] arrays: p is w's interface part, the interior part of w is
// overwritten with the extension, the result goes to q's interface rows.
template <typename T>
static int schur_apply(sgw_ctx* c, PrecT<T>& pr, const Tols& tl, T* w, T* q, hipStream_t st) {
  const int P = c->P, NF = c->NF, nI = c->nI, nG = c->nG;
  k::fill2d<T>(P, nI, w, NF, T(0), st);
  K1<T>(c, pr.G, &c->hal_G0, 0, nI, w, NF, pr.T1, NF, -1.0, 0.0, st);
  int rc = inner_solve<T>(c, pr.D, false, pr.T1, NF, w, NF, tl.inner, tl.inner_max_iter,
                          kSiteSchur, st);
  if (rc < 0) return rc;
  K1<T>(c, pr.G, &c->hal_GI, nI, nG, w, NF, q, NF, 1.0, 0.0, st);
  return rc;
}

// z_G = M_NNC^{-1} r_G (Eq. NNCP2).  The local residuals D_s R_s r on the
// remaining nodes drive one batched Neumann solve (corners held at zero);
// the coarse right-hand side d_c = sum_s B_c^T (D_s r_c - K~^s_{c,(ir)} y^s)
// gives u_c = F_cc^{-1} d_c (FP64); the remaining values get the coarse basis
// term Phi_s u_c^s (the second Neumann solve of Eq. urs, precomputed), and
// the weighted gather sum_s R_s^T D_s (...) assembles z (Eq. ugb).
template <typename T>
static int precond(sgw_ctx* c, PrecT<T>& pr, const Tols& tl, const T* r, T* z, hipStream_t st) {
  const int P = c->P, NF = c->NF, NT = c->NT, nG = c->nG;
  k::scatter_to_torn<T>(NT, P, c->torn_gidx, c->torn_w, r, NF, pr.Tt, NT, st);
  int rc = inner_solve<T>(c, pr.N, true, pr.Tt, NT, pr.Yt, NT, tl.precond, tl.inner_max_iter,
                          kSiteNeumann, st);
  if (rc < 0) return rc;
  if (c->nC > 0) {
    k::coarse_rhs<T>(c->co, r, NF, pr.Yt, NT, c->dc, st);
    k::coarse_solve(c->cf, c->dc, c->uc, sizeof(T) == 4, st);
    k::coarse_lift<T>(c->co, c->nsub, c->uc, pr.Yt, NT, st);
  }
  k::gather_from_torn<T>(nG, P, c->gam_ptr, c->gam_torn, c->gam_w, c->g2c, pr.Yt, NT, c->uc,
                         c->nC, z, NF, st);
  return rc;
}

// One SG system K~ U = F on the DD numbering (F, X full [P][NF] arrays of
// this precision); X holds the interface initial guess on entry (with
// zero_guess the guess is zero and X need not be set) and the full solution
// on exit.
template <typename T>
static int dd_solve(sgw_ctx* c, PrecT<T>& pr, const Tols& tl, const T* F, T* X, hipStream_t st,
                    int& outer_its, double& relres, const double* fallback = nullptr,
                    bool zero_guess = false) {
  const int P = c->P, NF = c->NF, nI = c->nI, nG = c->nG;
  int warn = 0, rc;
  // H2: condensation G = F_G - K~_GI K~_II^{-1} F_I
  rc = inner_solve<T>(c, pr.D, false, F, NF, pr.T1, NF, tl.inner, tl.inner_max_iter,
                      kSiteCondense, st);
  if (rc < 0) return rc;
  warn |= rc;
  k::fill2d<T>(P, nG, pr.T1 + nI, NF, T(0), st);
  k::copy2d<T, T>(P, nG, F + nI, NF, pr.Gv + nI, NF, 1.0, st);
  K1<T>(c, pr.G, &c->hal_GI, nI, nG, pr.T1, NF, pr.Gv, NF, -1.0, 1.0, st);
  // H5 without a final solve: every Schur apply S p leaves w = -K~_II^{-1}
  // K~_IG p in the interior part of its input vector (Pw), so the interior
  // solution U_I = K~_II^{-1} (F_I - K~_IG U_G) accumulates alongside the
  // interface iterate: U_I = K~_II^{-1} F_I + w(x0) + sum_k alpha_k w(p_k),
  // which is one update over all rows, X += alpha Pw.
  k::copy2d<T, T>(P, nI, pr.T1, NF, X, NF, 1.0, st);
  // The PCG scalars (alpha, beta, r'z) stay on the device; the host reads
  // r'r (and G'G at the start) for the stopping test, once per iteration.
  // Dot products over the interface rows give partial sums per (row chunk,
  // mode), NP = chunks x P of them, summed in a fixed order.  osc = [G'G
  // partials (NP)][r'r partials (NP)][ds: r'z by parity, alpha, beta,
  // breakdown flag, ...]
  const int gc = c->ngchunk, NP = gc * P;
  double* const ggp = c->osc;
  double* const rrp = c->osc + NP;
  double* const ds = c->osc + 2 * NP;
  auto read_rr = [&](double& rr, bool with_gg, double* gg) -> int {
    const int off = with_gg ? 0 : NP;
    HIPCHK(hipMemcpyAsync(c->hosc + off, c->osc + off, (2 * NP + 8 - off) * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    prof_stage(c, st);
    HIPCHK(hipStreamSynchronize(st));
    prof_harvest(c);
    rr = 0.0;
    for (int j = 0; j < NP; ++j) rr += c->hosc[NP + j];
    if (with_gg) {
      *gg = 0.0;
      for (int j = 0; j < NP; ++j) *gg += c->hosc[j];
    }
    return 0;
  };
  k::fill2d<double>(1, 8, ds, 8, 0.0, st);
  k::seg_dot<T>(gc, c->goff, P, pr.Gv + nI, NF, pr.Gv + nI, NF, ggp, nullptr, 0, nullptr, 0,
                nullptr, st);
  // H3/H4: PCG on S U_G = G, initial guess in X's interface part
  T* x = X + nI;
  T* r = pr.R + nI;
  T* z = pr.Z + nI;
  T* zp = pr.Zp + nI;
  T* p = pr.Pw + nI;
  T* q = pr.Qw + nI;
  if (zero_guess) {  // x0 = 0: r = G, no Schur apply
    k::fill2d<T>(P, nG, x, NF, T(0), st);
    k::copy2d<T, T>(P, nG, pr.Gv + nI, NF, r, NF, 1.0, st);
  } else {
    k::copy2d<T, T>(P, nG, x, NF, p, NF, 1.0, st);
    if ((rc = schur_apply<T>(c, pr, tl, pr.Pw, pr.Qw, st)) < 0) return rc;
    warn |= rc;
    k::axpby2d<T>(P, nG, 1.0, pr.Gv + nI, NF, -1.0, q, NF, r, NF, st);
    k::axpby2d<T>(P, nI, 1.0, X, NF, 1.0, pr.Pw, NF, X, NF, st);  // U_I += w(x0)
  }
  double gg = 0.0, rr = 0.0;
  if (fallback) {  // a learned guess worse than the zero guess is replaced
    double rr0;
    k::seg_dot<T>(gc, c->goff, P, r, NF, r, NF, rrp, nullptr, 0, nullptr, 0, nullptr, st);
    if ((rc = read_rr(rr0, true, &gg))) return rc;
    if (!(rr0 <= gg)) {
      k::axpby2d<T>(P, nI, 1.0, X, NF, -1.0, pr.Pw, NF, X, NF, st);  // U_I -= w(x0)
      k::copy2d<T, double>(P, nG, fallback, nG, x, NF, 1.0, st);
      k::copy2d<T, T>(P, nG, x, NF, p, NF, 1.0, st);
      if ((rc = schur_apply<T>(c, pr, tl, pr.Pw, pr.Qw, st)) < 0) return rc;
      warn |= rc;
      k::axpby2d<T>(P, nG, 1.0, pr.Gv + nI, NF, -1.0, q, NF, r, NF, st);
      k::axpby2d<T>(P, nI, 1.0, X, NF, 1.0, pr.Pw, NF, X, NF, st);
      c->guess_fallbacks++;
    }
  }
  if ((rc = precond<T>(c, pr, tl, r, z, st)) < 0) return rc;
  warn |= rc;
  k::copy2d<T, T>(P, nG, z, NF, p, NF, 1.0, st);
  int par = 0;
  k::seg_dot<T>(gc, c->goff, P, r, NF, z, NF, c->part, r, NF, r, NF, rrp, st);
  k::outer_scalars(0, NP, c->part, nullptr, ds, par, st);
  if ((rc = read_rr(rr, true, &gg))) return rc;
  const double stop2 = tl.rtol * tl.rtol * gg;
  // flexible CG (Polak-Ribiere beta): the preconditioner's Neumann solves run
  // to their own tolerance, so M^{-1} may vary slightly between iterations;
  // with an exact preconditioner this is the classic PCG recurrence
  int it = 0;
  while (rr > stop2 && gg > 0.0) {
    if (it >= tl.max_iter) {
      warn = SGW_NOT_CONVERGED;
      break;
    }
    if ((rc = schur_apply<T>(c, pr, tl, pr.Pw, pr.Qw, st)) < 0) return rc;
    warn |= rc;
    k::seg_dot<T>(gc, c->goff, P, p, NF, q, NF, c->part, nullptr, 0, nullptr, 0, nullptr, st);
    k::outer_scalars(1, NP, c->part, nullptr, ds, par, st);
    k::axpby2d_dev<T>(P, NF, 1.0, -1, X, NF, 1.0, 2, pr.Pw, NF, X, NF, ds, st);  // U += alpha Pw
    k::axpby2d_dev<T>(P, nG, 1.0, -1, r, NF, -1.0, 2, q, NF, r, NF, ds, st);
    ++it;
    k::seg_dot<T>(gc, c->goff, P, r, NF, r, NF, rrp, nullptr, 0, nullptr, 0, nullptr, st);
    if ((rc = read_rr(rr, false, nullptr))) return rc;
    if (c->hosc[2 * NP + 4] != 0.0) {
      c->err = "breakdown (p'Sp <= 0) in the interface PCG";
      return c->hosc[2 * NP + 4] == 1.0 ? SGW_EBREAKDOWN : SGW_ENAN;
    }
    if (!std::isfinite(rr)) {
      c->err = "non-finite interface residual";
      return SGW_ENAN;
    }
    if (rr <= stop2) break;
    std::swap(z, zp);  // zp = the previous preconditioned residual
    if ((rc = precond<T>(c, pr, tl, r, z, st)) < 0) return rc;
    warn |= rc;
    k::seg_dot<T>(gc, c->goff, P, r, NF, z, NF, c->part, r, NF, zp, NF, c->part2, st);
    k::outer_scalars(2, NP, c->part, c->part2, ds, par, st);
    k::axpby2d_dev<T>(P, nG, 1.0, -1, z, NF, 1.0, 3, p, NF, p, NF, ds, st);
    par ^= 1;
  }
  outer_its = it;
  relres = gg > 0.0 ? std::sqrt(rr / gg) : 0.0;
  return warn ? SGW_NOT_CONVERGED : 0;
}

// ---------------------------------------------------------------------------
// mesh-node <-> DD-numbering conversions and moments
// ---------------------------------------------------------------------------
__global__ void k_mesh_to_dd(int P, int NF, int nn, const int* dd2mesh, const double* src,
                             double* dst) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * NF) return;
  int j = (int)(t / NF), dd = (int)(t % NF);
  dst[(size_t)j * NF + dd] = src[(size_t)j * nn + dd2mesh[dd]];
}
__global__ void k_dd_to_mesh(int P, int NF, int nn, const int* dd2mesh, const double* src,
                             double* dst) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * NF) return;
  int j = (int)(t / NF), dd = (int)(t % NF);
  dst[(size_t)j * nn + dd2mesh[dd]] = src[(size_t)j * NF + dd];
}
// H10: mean = mode 0, var = sum_{j>=1} u_j^2 (normalised basis)
__global__ void k_moments(int P, int NF, const int* dd2mesh, const double* U, double* mean,
                          double* var) {
  int dd = blockIdx.x * blockDim.x + threadIdx.x;
  if (dd >= NF) return;
  double v = 0.0;
  for (int j = 1; j < P; ++j) {
    double u = U[(size_t)j * NF + dd];
    v += u * u;
  }
  int m = dd2mesh[dd];
  if (mean) mean[m] = U[dd];
  if (var) var[m] = v;
}
__global__ void k_diag_scale(long long N, int NF, const double* diag, const double* r, double* z) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  z[t] = r[t] / diag[t % NF];
}

static int to_dd(sgw_ctx* c, const double* src, int where, double* dst, hipStream_t st) {
  const size_t bytes = (size_t)c->P * c->nn * sizeof(double);
  const double* s = src;
  if (where == SGW_HOST) {
    HIPCHK(hipMemcpyAsync(c->meshbuf, src, bytes, hipMemcpyHostToDevice, st));
    s = c->meshbuf;
  }
  long long N = (long long)c->P * c->NF;
  k_mesh_to_dd<<<(int)((N + 255) / 256), 256, 0, st>>>(c->P, c->NF, c->nn, c->dd2mesh, s, dst);
  return 0;
}

static int from_dd(sgw_ctx* c, const double* src, double* dst, int where, hipStream_t st) {
  const size_t bytes = (size_t)c->P * c->nn * sizeof(double);
  double* t = where == SGW_HOST ? c->meshbuf : dst;
  HIPCHK(hipMemsetAsync(t, 0, bytes, st));
  long long N = (long long)c->P * c->NF;
  k_dd_to_mesh<<<(int)((N + 255) / 256), 256, 0, st>>>(c->P, c->NF, c->nn, c->dd2mesh, src, t);
  if (where == SGW_HOST) {
    HIPCHK(hipMemcpyAsync(dst, t, bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return 0;
}

// (I (x) M) A = rhs by Jacobi-preconditioned CG over all modes (set-up only).
static int mass_solve(sgw_ctx* c, const double* rhs, double* out, hipStream_t st) {
  const int P = c->P, NF = c->NF;
  const long long N = (long long)P * NF;
  double* r = c->d64.R;
  double* z = c->d64.Z;
  double* p = c->d64.Pw;
  double* q = c->d64.Qw;
  k::fill2d<double>(P, NF, out, NF, 0.0, st);
  k::copy2d<double, double>(P, NF, rhs, NF, r, NF, 1.0, st);
  auto dot = [&](const double* a, const double* b, double& v) -> int {
    k::seg_dot<double>(1, c->alloff, P, a, NF, b, NF, c->part, nullptr, 0, nullptr, 0, nullptr, st);
    std::vector<double> h(P);
    HIPCHK(hipMemcpyAsync(h.data(), c->part, P * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    v = 0.0;
    for (double x : h) v += x;
    return 0;
  };
  int rc;
  double bb, rz, rr;
  if ((rc = dot(r, r, bb))) return rc;
  if (bb == 0.0) return 0;
  k_diag_scale<<<(int)((N + 255) / 256), 256, 0, st>>>(N, NF, c->mdiag, r, z);
  k::copy2d<double, double>(P, NF, z, NF, p, NF, 1.0, st);
  if ((rc = dot(r, z, rz))) return rc;
  rr = bb;
  for (int it = 0; it < 500 && rr > 1e-30 * bb; ++it) {
    k::mass_apply<double>(c->d64.G, 0, NF, P, p, NF, q, NF, 1.0, 0.0, st);
    double pq;
    if ((rc = dot(p, q, pq))) return rc;
    double al = rz / pq;
    k::axpby2d<double>(P, NF, 1.0, out, NF, al, p, NF, out, NF, st);
    k::axpby2d<double>(P, NF, 1.0, r, NF, -al, q, NF, r, NF, st);
    if ((rc = dot(r, r, rr))) return rc;
    k_diag_scale<<<(int)((N + 255) / 256), 256, 0, st>>>(N, NF, c->mdiag, r, z);
    double rzn;
    if ((rc = dot(r, z, rzn))) return rc;
    k::axpby2d<double>(P, NF, 1.0, z, NF, rzn / rz, p, NF, p, NF, st);
    rz = rzn;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// coarse set-up kernels: for local corner slot lcl and mode m, the right-hand
// side -K~^s_{(ir),c} e_(c,m) of every subdomain that has that corner, and,
// from the Neumann solution x, the coarse basis Phi_s[:, (m,lcl)] (remaining
// rows) and the local coarse-matrix column
// F^s[(m',lc'), (m,lcl)] = K~^s_cc + K~^s_{c',(ir)} x  (Eq. Fcc_2 with
// S_cc - S_cr S_rr^{-1} S_rc written as one Neumann solve).
// ---------------------------------------------------------------------------
__global__ void k_basis_rhs(k::DCoarse co, int lcl, int m, double* bt, int ldt) {
  int s = blockIdx.x;
  int ncs = co.sc_ptr[s + 1] - co.sc_ptr[s];
  if (lcl >= ncs) return;
  int lc = co.sc_ptr[s] + lcl;
  int ne = co.cc_ptr[lc + 1] - co.cc_ptr[lc];
  for (int t = threadIdx.x; t < ne * co.P; t += blockDim.x) {
    int e = co.cc_ptr[lc] + t / co.P, j = t % co.P;
    const double* kv = co.cc_val + (size_t)e * co.nk;
    double acc = 0.0;
    for (int g = co.gi_ptr[j]; g < co.gi_ptr[j + 1]; ++g)
      if (co.gi_j[g] == m) acc += co.gi_v[g] * kv[co.gi_k[g]];
    bt[(size_t)j * ldt + co.cc_torn[e]] = -acc;
  }
}

__global__ void k_basis_store(k::DCoarse co, int lcl, int m, const double* xt, int ldt,
                              double* fs) {
  int s = blockIdx.x;
  int lc0 = co.sc_ptr[s], ncs = co.sc_ptr[s + 1] - lc0;
  if (lcl >= ncs) return;
  int nrem = co.rem_off[s + 1] - co.rem_off[s];
  long long nout = (long long)co.P * nrem;
  double* ph = const_cast<double*>(co.phi) + co.phi_off[s] + ((size_t)m * ncs + lcl) * nout;
  for (long long o = threadIdx.x; o < nout; o += blockDim.x) {
    int j = (int)(o / nrem), tr = (int)(o % nrem);
    ph[o] = xt[(size_t)j * ldt + co.rem_list[co.rem_off[s] + tr]];
  }
  const int MP = co.maxc * co.P;
  double* F = fs + (size_t)s * MP * MP;
  for (int t = threadIdx.x; t < ncs * co.P; t += blockDim.x) {
    int l2 = t / co.P, m2 = t % co.P;
    int lc = lc0 + l2;
    double v = 0.0;  // the K~^s_cc term is added on the host
    for (int e = co.cc_ptr[lc]; e < co.cc_ptr[lc + 1]; ++e) {
      const double* kv = co.cc_val + (size_t)e * co.nk;
      int row = co.cc_torn[e];
      for (int g = co.gi_ptr[m2]; g < co.gi_ptr[m2 + 1]; ++g)
        v += co.gi_v[g] * kv[co.gi_k[g]] * xt[(size_t)co.gi_j[g] * ldt + row];
    }
    F[(size_t)(m2 * co.maxc + l2) * MP + (m * co.maxc + lcl)] = v;
  }
}

// Device state of one precision: operator values (FP32 copies for the
// refinement path), system workspaces and interface vectors.
// Natural (lexicographic mesh) order of the rows of every block of a
// subdomain system: crow[r0 + i] = system row at position i of block
// [r0, r1), cnb[8 (r0 + i) + s] = block-local position of that row's slot-s
// neighbour (slots past the matrix width: the row itself).  mesh_of(row)
// gives a row's mesh node.  crow_h keeps the host copy of crow.
template <class MeshOf>
static void natural_order(sgw_ctx* c, const Ell& E, const std::vector<int>& off, MeshOf mesh_of,
                          const int** crow_d, const unsigned short** cnb_d,
                          std::vector<int>& crow_h) {
  const int NR = E.nrows, n1 = c->h.n + 1;
  std::vector<int> crow(NR > 0 ? NR : 1), pos(NR > 0 ? NR : 1);
  std::vector<unsigned short> cnb((size_t)8 * std::max(NR, 1), 0);
  for (size_t b = 0; b + 1 < off.size(); ++b) {
    const int r0 = off[b], r1 = off[b + 1];
    std::vector<int> rows;
    for (int r = r0; r < r1; ++r) rows.push_back(r);
    std::sort(rows.begin(), rows.end(), [&](int a, int q) {
      const int va = mesh_of(a), vq = mesh_of(q);
      return std::make_pair(va / n1, va % n1) < std::make_pair(vq / n1, vq % n1);
    });
    for (int i = 0; i < r1 - r0; ++i) {
      crow[r0 + i] = rows[i];
      pos[rows[i]] = i;
    }
  }
  for (size_t b = 0; b + 1 < off.size(); ++b)
    for (int i = off[b]; i < off[b + 1]; ++i)
      for (int s = 0; s < 8; ++s)
        cnb[(size_t)8 * i + s] =
            (unsigned short)(s < std::min(E.W, 7) ? pos[E.col[(size_t)s * NR + crow[i]]]
                                                  : i - off[b]);
  *crow_d = upload(c, crow);
  *cnb_d = upload(c, cnb);
  crow_h = crow;
}

// Row-group halos of an ELL matrix for rows [r0, nrows) (see k::DHalo):
// plain 64-row chunks, or (boff = block offsets of a block-diagonal system,
// r0 = 0) chunks of at most 64 rows that never straddle a block.
static k::DHalo build_halo(sgw_ctx* c, const Ell& E, int r0,
                           const std::vector<int>* boff = nullptr) {
  k::DHalo H;
  const int nr = std::max(E.nrows - r0, 0);
  H.r0 = r0;
  H.nr = nr;
  std::vector<int> grow, gblk, bgrp;
  if (boff) {
    H.aligned64 = false;
    for (size_t b = 0; b + 1 < boff->size(); ++b) {
      bgrp.push_back((int)grow.size());
      for (int a = (*boff)[b]; a < (*boff)[b + 1]; a += 64) {
        grow.push_back(a);
        gblk.push_back((int)b);
      }
    }
    bgrp.push_back((int)grow.size());
  } else {
    for (int a = r0; a < E.nrows; a += 64) grow.push_back(a);
  }
  H.ng = (int)grow.size();
  grow.push_back(E.nrows);
  std::vector<int> ptr{0}, idx, cols;
  std::vector<unsigned short> lcol((size_t)E.W * std::max(nr, 1), 0);
  for (int g = 0; g < H.ng; ++g) {
    const int a = grow[g], b = grow[g + 1];
    cols.clear();
    for (int s = 0; s < E.W; ++s)
      for (int r = a; r < b; ++r) cols.push_back(E.col[(size_t)s * E.nrows + r]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int s = 0; s < E.W; ++s)
      for (int r = a; r < b; ++r) {
        const int cc = E.col[(size_t)s * E.nrows + r];
        lcol[(size_t)s * nr + (r - r0)] =
            (unsigned short)(std::lower_bound(cols.begin(), cols.end(), cc) - cols.begin());
      }
    idx.insert(idx.end(), cols.begin(), cols.end());
    ptr.push_back((int)idx.size());
    H.hmax = std::max(H.hmax, (int)cols.size());
  }
  if (idx.empty()) idx.push_back(0);
  H.ptr = upload(c, ptr);
  H.idx = upload(c, idx);
  H.lcol = upload(c, lcol);
  H.grow = upload(c, grow);
  if (boff) {
    H.gblk = upload(c, gblk.empty() ? std::vector<int>{0} : gblk);
    H.bgrp = upload(c, bgrp);
  }
  return H;
}

template <typename T>
static void setup_prec(sgw_ctx* c, PrecT<T>& pr, bool refine) {
  const Host& h = c->h;
  const int P = c->P;
  auto ell = [&](const Ell& E) {
    k::DEll<T> d;
    d.nrows = E.nrows;
    d.W = E.W;
    d.nk = E.nk;
    d.col = upload(c, E.col);
    if constexpr (sizeof(T) == 8) {
      d.val = upload(c, E.val);
      d.mval = upload(c, E.mval);
    } else {
      d.val = upload(c, to_f(E.val));
      d.mval = upload(c, to_f(E.mval));
    }
    return d;
  };
  pr.G = ell(h.glob);
  pr.D.A = ell(h.dir);
  pr.N.A = ell(h.neu);
  if constexpr (sizeof(T) == 8) {
    pr.D.F = upload_factor(c, h.fD);
    pr.N.F = upload_factor(c, h.fN);
  } else {
    pr.D.F = c->d64.D.F;  // one factor upload holds both precisions
    pr.N.F = c->d64.N.F;
  }
  pr.D.nrows = h.nI;
  pr.D.nb = h.nsub;
  pr.D.row_off = pr.D.F.row_off;
  pr.N.nrows = h.NT;
  pr.N.nb = h.nsub;
  pr.N.row_off = pr.N.F.row_off;
  auto pickq = [&](const k::DFactor& f) {
    int ntiles = (P + 7) / 8;
    int q = (P + ntiles - 1) / ntiles;
    while (q > 1 && k::tri_lds_bytes<T>(f, q) > 150 * 1024) --q;
    return q;
  };
  pr.D.Q = pickq(pr.D.F);
  pr.N.Q = pickq(pr.N.F);
  // Chebyshev preconditioner: step coefficients of every block (from its
  // spectral interval, in double, then rounded to T), largest block
  auto coefs = [&](const std::vector<double>& iv) {
    const int deg = c->cheb_deg, nb = (int)(iv.size() / 2);
    std::vector<double> cd(2 * (size_t)deg);
    std::vector<T> cc(std::max<size_t>(2 * (size_t)deg * nb, 1), T(0));
    for (int b = 0; b < nb; ++b) {
      k::cheb_coefficients(iv[2 * b], iv[2 * b + 1], deg, cd.data());
      for (int e = 0; e < 2 * deg; ++e) cc[(size_t)b * 2 * deg + e] = (T)cd[e];
    }
    return upload(c, cc);
  };
  pr.D.cheb_cc = coefs(h.chebD);
  pr.N.cheb_cc = coefs(h.chebN);
  auto maxblk = [&](const std::vector<int>& off) {
    int m = 0;
    for (size_t b = 0; b + 1 < off.size(); ++b) m = std::max(m, off[b + 1] - off[b]);
    return m;
  };
  pr.D.max_block_rows = maxblk(h.Ioff);
  pr.N.max_block_rows = maxblk(h.Toff);
  pr.D.halo = &c->hal_D;
  pr.N.halo = &c->hal_N;
  // largest blocks first (longest-processing-time order for the per-block
  // kernels; matters for uneven partitions)
  auto lpt = [&](const std::vector<int>& off) {
    std::vector<int> o(off.size() - 1);
    for (size_t b = 0; b < o.size(); ++b) o[b] = (int)b;
    std::stable_sort(o.begin(), o.end(), [&](int a, int q) {
      return off[a + 1] - off[a] > off[q + 1] - off[q];
    });
    return o;
  };
  if constexpr (sizeof(T) == 8) {
    pr.D.lpt = upload(c, lpt(h.Ioff));
    pr.N.lpt = upload(c, lpt(h.Toff));
    pr.D.F.order = pr.D.lpt;
    pr.N.F.order = pr.N.lpt;
  } else {
    pr.D.lpt = c->d64.D.lpt;
    pr.N.lpt = c->d64.N.lpt;
  }
  if constexpr (sizeof(T) == 8) {
    natural_order(c, h.dir, h.Ioff, [&](int r) { return h.dd2mesh[r]; }, &pr.D.crow, &pr.D.cnb,
                  c->crow_h[0]);
    natural_order(c, h.neu, h.Toff, [&](int r) { return h.dd2mesh[h.torn2dd[r]]; }, &pr.N.crow,
                  &pr.N.cnb, c->crow_h[1]);
  } else {
    pr.D.crow = c->d64.D.crow;
    pr.D.cnb = c->d64.D.cnb;
    pr.N.crow = c->d64.N.crow;
    pr.N.cnb = c->d64.N.cnb;
  }
  // the mean-matrix rows (coefficient slot k = 0) in natural order, as
  // [8]-records of this precision
  auto pack_mean = [&](const Ell& E, const std::vector<int>& crow) {
    const int NR = E.nrows, W = std::min(E.W, 7);
    std::vector<T> cv((size_t)8 * std::max(NR, 1), T(0));
    for (int i = 0; i < NR; ++i)
      for (int s = 0; s < W; ++s) cv[(size_t)8 * i + s] = (T)E.val[(size_t)s * NR + crow[i]];
    return upload(c, cv);
  };
  pr.D.cval = pack_mean(h.dir, c->crow_h[0]);
  pr.N.cval = pack_mean(h.neu, c->crow_h[1]);
  for (SysT<T>* S : {&pr.D, &pr.N}) {
    const int qmax = std::max(1, k::cheb_max_q<T>(S->max_block_rows, 0));
    int ntiles = (P + qmax - 1) / qmax;
    int q = (P + ntiles - 1) / ntiles;
    while (q > 1 && k::cheb_lds_bytes<T>(S->max_block_rows, q, 0) > 150 * 1024) --q;
    S->cq = q;
    S->cshape = 0;
  }
  const sgw_problem_desc& d = h.d;
  double loose = refine ? d.ir_precond_rtol : d.precond_rtol;
  double tight = refine ? d.ir_inner_rtol : d.inner_rtol;
  if (loose > tight) pr.N.loose_tol = loose;
  for (SysT<T>* S : {&pr.D, &pr.N}) {
    size_t n = (size_t)P * S->nrows;
    S->x = dalloc<T>(c, n);
    S->r = dalloc<T>(c, n);
    S->z = dalloc<T>(c, n);
    S->p = dalloc<T>(c, n);
    S->q = dalloc<T>(c, n);
    S->p2 = dalloc<T>(c, n);
  }
  size_t nv = (size_t)P * h.NF;
  for (T** v : {&pr.X, &pr.R, &pr.Z, &pr.Zp, &pr.Pw, &pr.Qw, &pr.T1, &pr.Gv}) *v = dalloc<T>(c, nv);
  if (refine) {
    pr.Fb = dalloc<T>(c, nv);
    pr.Xb = dalloc<T>(c, nv);
  }
  pr.Tt = dalloc<T>(c, (size_t)P * h.NT);
  pr.Yt = dalloc<T>(c, (size_t)P * h.NT);
  pr.ready = true;
}

// X64 += (double) D32 over [P][NF]
__global__ void k_add_f32(long long N, double* x, const float* d, double scale) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) x[t] += scale * (double)d[t];
}

// Dot products over all rows of full [P][NF] arrays (FP64 sums over row
// chunks and modes, fixed order): out = a'b and, with c and d, out2 = c'd,
// read with one synchronisation
template <typename T>
static int fdot(sgw_ctx* c, const T* a, const T* b, double& out, hipStream_t st,
                const T* cc = nullptr, const T* dd = nullptr, double* out2 = nullptr) {
  const int P = c->P, nc = c->nfchunk;
  const size_t np = (size_t)nc * P;
  k::seg_dot<T>(nc, c->fchunk, P, a, c->NF, b, c->NF, c->part, cc, c->NF, dd, c->NF,
                cc ? c->part2 : nullptr, st);
  HIPCHK(hipMemcpyAsync(c->hpart, c->part, np * sizeof(double), hipMemcpyDeviceToHost, st));
  if (cc)
    HIPCHK(hipMemcpyAsync(c->hpart + np, c->part2, np * sizeof(double), hipMemcpyDeviceToHost,
                          st));
  prof_stage(c, st);
  HIPCHK(hipStreamSynchronize(st));
  prof_harvest(c);
  out = 0.0;
  for (size_t e = 0; e < np; ++e) out += c->hpart[e];
  if (cc) {
    *out2 = 0.0;
    for (size_t e = 0; e < np; ++e) *out2 += c->hpart[np + e];
  }
  return 0;
}

// Whether a step carries the images K~ U, K~ V, K~ A along with the state:
// in the refinement path with stiffness damping, where the effective force
// needs K~ Uc (Eq. fparts) and the solve's final FP64 residual R = F - K~ U1
// already holds K~ of the new state.
static bool carry_images(const sgw_problem_desc& d) {
  return d.precision == SGW_FP32_IR64 && d.alpha1 != 0.0;
}

// H7: FP64 iterative refinement around the FP32 DD-PCG.  The residual
// R = F - K~ X and the update X += D are FP64 on the global SG system; each
// correction K~ D = R is solved by the whole DD method in FP32 (coarse grid
// FP64) to the relative tolerances below.  Stops when ||R|| <= rtol ||F||.
//
// x0 (optional): X holds U + x0[0] V + x0[1] A of the carried state, whose
// images give the first residual without an SG apply; every later residual,
// and so the accepted one, is formed by the FP64 apply.
static int ir_solve(sgw_ctx* c, const double* F, double* X, hipStream_t st, int& outer_total,
                    int& sweeps, double& relres, const double* fallback = nullptr,
                    const double* x0 = nullptr) {
  const sgw_problem_desc& d = c->h.d;
  const int P = c->P, NF = c->NF;
  PrecT<float>& pr = c->f32;
  double* R = c->d64.R;
  Tols tl{d.ir_outer_rtol, d.ir_inner_rtol, d.ir_precond_rtol, d.max_iter, d.inner_max_iter};
  double ff = 0.0;
  int rc = 0;
  int warn = 0;
  outer_total = 0;
  sweeps = 0;
  for (bool first = true;; first = false) {
    if (first && x0) {
      k::residual_images(P, NF, F, c->GU, c->GV, c->GA, x0[0], x0[1], R, st);
    } else {
      k::copy2d<double, double>(P, NF, F, NF, R, NF, 1.0, st);
      K1<double>(c, c->d64.G, &c->hal_G0, 0, NF, X, NF, R, NF, -1.0, 1.0, st);
    }
    double rr;
    if (first) rc = fdot<double>(c, R, R, rr, st, F, F, &ff);  // with F'F
    else rc = fdot<double>(c, R, R, rr, st);
    if (rc) return rc;
    relres = ff > 0.0 ? std::sqrt(rr / ff) : 0.0;
    if (fallback && sweeps == 0 && !(rr <= ff)) {
      // a learned interface guess worse than the zero guess: Newmark instead
      k::copy2d<double, double>(P, c->nG, fallback, c->nG, X + c->nI, NF, 1.0, st);
      c->guess_fallbacks++;
      fallback = nullptr;
      continue;
    }
    if (!std::isfinite(rr)) {
      c->err = "non-finite refinement residual";
      return SGW_ENAN;
    }
    if (rr <= d.rtol * d.rtol * ff) break;
    if (sweeps >= kIrMaxSweeps) {
      warn = SGW_NOT_CONVERGED;
      break;
    }
    // the correction equation is solved for the residual scaled to unit RMS,
    // which keeps the FP32 values away from the ends of their range
    const double scale = std::sqrt(rr / ((double)P * NF));
    k::copy2d<float, double>(P, NF, R, NF, pr.Fb, NF, 1.0 / scale, st);
    int its = 0;
    double rel32 = 0.0;
    rc = dd_solve<float>(c, pr, tl, pr.Fb, pr.Xb, st, its, rel32, nullptr, true);
    if (rc < 0) return rc;
    warn |= rc;
    outer_total += its;
    long long N = (long long)P * NF;
    k_add_f32<<<(int)((N + 255) / 256), 256, 0, st>>>(N, X, pr.Xb, scale);
    ++sweeps;
  }
  return warn ? SGW_NOT_CONVERGED : 0;
}


// Every device array a kernel may touch must exist before create returns
// (a missing allocation is reported instead of reaching a kernel).
template <typename T>
static bool prec_complete(const PrecT<T>& pr, bool refine) {
  const void* ps[] = {pr.G.col, pr.G.val, pr.G.mval, pr.D.A.col, pr.D.A.val, pr.N.A.col,
                      pr.N.A.val, pr.D.x, pr.D.r, pr.D.z, pr.D.p, pr.D.q, pr.N.x, pr.N.r,
                      pr.N.z, pr.N.p, pr.N.q, pr.X, pr.R, pr.Z, pr.Zp, pr.Pw, pr.Qw, pr.T1,
                      pr.Gv, pr.Tt, pr.Yt, pr.D.row_off, pr.N.row_off, pr.D.crow, pr.D.cnb,
                      pr.N.crow, pr.N.cnb, pr.D.cheb_cc, pr.N.cheb_cc, pr.D.cval, pr.N.cval,
                      pr.D.p2, pr.N.p2};
  for (const void* p : ps)
    if (!p) return false;
  return !refine || (pr.Fb && pr.Xb);
}

static bool check_pointers(sgw_ctx* c) {
  const void* ps[] = {c->U, c->V, c->A, c->Um, c->Uc, c->Wm, c->F, c->hist, c->gnew, c->smax,
                      c->mx, c->my, c->pqg, c->meshbuf, c->meshbuf2,
                      c->part, c->part2, c->osc, c->sc, c->flags, c->goff, c->alloff,
                      c->fchunk,
                      c->dd2mesh,
                      c->mdiag, c->torn_gidx, c->torn_w, c->gam_ptr, c->gam_torn, c->gam_w,
                      c->g2c, c->dc, c->uc, c->phi, c->gt.mask, c->gt.pair_beg, c->gt.ent_beg,
                      c->gt.pair_cnt, c->gt.ent_i, c->gt.ent_c, c->gt.ent_cf};
  for (const void* p : ps)
    if (!p) {
      c->err = "internal error: a device array was not allocated";
      return false;
    }
  if (carry_images(c->h.d) && (!c->GU || !c->GV || !c->GA)) {
    c->err = "internal error: a device array was not allocated";
    return false;
  }
  if (!prec_complete(c->d64, false) ||
      (c->h.d.precision == SGW_FP32_IR64 && (!prec_complete(c->f32, true) || !c->phih))) {
    c->err = "internal error: a device array of a solver precision was not allocated";
    return false;
  }
  return true;
}
// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sgw_last_error(const sgw_ctx* c) { return c ? c->err.c_str() : "null context"; }

int sgw_guess_record(sgw_ctx* c, float* X, float* T, long long capacity) {
  if (!c || capacity < 0 || ((X == nullptr) != (T == nullptr)) || (X && capacity == 0))
    return SGW_EINVAL;
  c->rec_x = X;
  c->rec_t = T;
  c->rec_cap = X ? capacity : 0;
  c->rec_n = 0;
  return 0;
}

int sgw_set_guess_model(sgw_ctx* c, sgw_mlp* m) {
  if (!c) return SGW_EINVAL;
  if (m && (m->nin != 4 || m->ng != 1)) {
    c->err = "the guess network must map 4 inputs to 1 output";
    return SGW_EINVAL;
  }
  c->mlp = m;
  return 0;
}

int sgw_set_guess(sgw_ctx* c, int mode) {
  if (!c) return SGW_EINVAL;
  if (mode != SGW_GUESS_PREV && mode != SGW_GUESS_NEWMARK && mode != SGW_GUESS_LEARNED) {
    c->err = "unknown guess mode";
    return SGW_EINVAL;
  }
  c->h.d.guess = mode;
  return 0;
}

long long sgw_query(const sgw_ctx* c, int what) {
  if (!c) return -1;
  switch (what) {
    case 0: return c->P;
    case 1: return c->nk;
    case 2: return c->NF;
    case 3: return c->nG;
    case 4: return c->nC;
    case 5: return c->nsub;
    case 6: return c->nn;
    case 7: return c->rec_n;
    case 8: return c->guess_fallbacks;
    case 9: return c->graph_launches;
    case 10: return c->gs_n;
    default: return -1;
  }
}

int sgw_profile(sgw_ctx* c, int enable) {
  if (!c || enable < 0) return SGW_EINVAL;
  prof_harvest(c);
  c->prof = enable != 0;
  c->prof_every = std::max(1, enable);
  if (c->acct && hipMemcpy(c->acct_h, c->acct, 4 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost) == hipSuccess)
    for (int q = 0; q < 4; ++q) c->acct_seen[q] = c->acct_h[q];
  for (int k2 = 0; k2 < 6; ++k2) {
    c->pcnt[k2] = 0;
    c->pms[k2] = 0.0;
    c->pbytes[k2] = 0.0;
    c->pseen[k2] = 0;
  }
  return 0;
}

int sgw_profile_read(sgw_ctx* c, int kind, long long* launches, double* ms, double* bytes) {
  if (!c || kind < 0 || kind > 5) return SGW_EINVAL;
  prof_harvest(c);
  if (launches) *launches = c->pcnt[kind];
  if (ms) *ms = c->pms[kind];
  if (bytes) *bytes = c->pbytes[kind];
  return 0;
}

// Autotuner: times the candidate launch shapes on the context's own data and
// keeps the fastest (mode tile of the triangular solves per system, SG-apply
// kernel with the unrolled tensor vs the table-driven one).
int sgw_autotune(sgw_ctx* c, void* stream, double* report, int nreport) {
  if (!c || nreport < 0) return SGW_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int kReport = 72;
  std::vector<double> rep(kReport, -1.0);
  const int reps = 10;
  auto time_it = [&](auto&& fn) -> double {
    fn();
    fn();
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i) fn();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return 1e3 * ms / reps;  // microseconds per launch
  };
  // mode tiles of one system: triangular solve (report at tri) and Chebyshev
  // (report at cheb); the preconditioner the context uses decides which one
  // is timed
  auto tune_sys = [&](auto& S, int tri, int cheb, int shape_slot) {
    using T = std::remove_reference_t<decltype(*S.r)>;
    k::fill2d<T>(c->P, S.nrows, S.r, S.nrows, T(1), st);
    double best = 1e300;
    if (c->inner_prec == SGW_INNER_CHEBYSHEV) {
      int bestq = S.cq, bests = S.cshape;
      for (int shape = 0; shape < 3; ++shape)
        for (int q = 1; q <= 8; ++q) {
          if (q > c->P || q > k::cheb_max_q<T>(S.max_block_rows, shape) ||
              k::cheb_lds_bytes<T>(S.max_block_rows, q, shape) > 150 * 1024)
            continue;
          double us = time_it([&] {
            (void)k::cheb_apply<T>(S.cval, S.row_off, S.lpt, S.crow, S.cnb, S.cheb_cc, S.nb, c->P,
                                   c->cheb_deg, q, shape, S.max_block_rows, S.r, S.nrows, S.z,
                                   S.nrows, c->part, c->part2, nullptr, 0, 0.0, nullptr,
                                   nullptr, nullptr, st);
          });
          if (rep[cheb + q - 1] < 0.0 || us < rep[cheb + q - 1]) rep[cheb + q - 1] = us;
          if (us < best) {
            best = us;
            bestq = q;
            bests = shape;
          }
        }
      S.cq = bestq;
      S.cshape = bests;
      rep[shape_slot] = bests;
    } else {
      int bestq = S.Q;
      for (int q = 1; q <= 8; ++q) {
        if (q > c->P || k::tri_lds_bytes<T>(S.F, q) > 150 * 1024) continue;
        double us = time_it([&] {
          k::tri_solve<T>(S.F, q, S.r, S.nrows, S.z, S.nrows, 1, 0, 0, st);
        });
        rep[tri + q - 1] = us;
        if (us < best) {
          best = us;
          bestq = q;
        }
      }
      S.Q = bestq;
    }
  };
  tune_sys(c->d64.D, 0, 18, 68);
  tune_sys(c->d64.N, 8, 26, 69);
  if (c->f32.ready) {
    tune_sys(c->f32.D, 34, 50, 70);
    tune_sys(c->f32.N, 42, 58, 71);
  }
  {
    // generated (unrolled tensor, staged x) vs table-driven SG apply on the
    // Dirichlet system, in FP64 and (refinement path) FP32; the precision the
    // steps run in decides
    const bool keep = c->gt.use_spec;
    double us[4] = {-1.0, -1.0, -1.0, -1.0};
    for (int v = 0; v < 2; ++v) {
      c->gt.use_spec = v == 0;
      SysT<double>& S = c->d64.D;
      us[v] = time_it([&] {
        k::sg_apply<double>(S.A, c->gt, S.halo, 0, S.nrows, S.r, S.nrows, S.q, S.nrows, 1.0, 0.0,
                            1, 0, 0, st);
      });
      if (c->f32.ready) {
        SysT<float>& F = c->f32.D;
        us[2 + v] = time_it([&] {
          k::sg_apply<float>(F.A, c->gt, F.halo, 0, F.nrows, F.r, F.nrows, F.q, F.nrows, 1.0f,
                             0.0f, 1, 0, 0, st);
        });
      }
    }
    rep[16] = us[0];
    rep[17] = us[1];
    rep[66] = us[2];
    rep[67] = us[3];
    c->gt.use_spec = keep && (c->f32.ready ? us[2] <= us[3] : us[0] <= us[1]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (hipGetLastError() != hipSuccess) {
    c->err = "kernel launch failed during autotuning";
    return SGW_EHIP;
  }
  if (report)
    for (int i = 0; i < nreport && i < kReport; ++i) report[i] = rep[i];
  return 0;
}

int sgw_set_cheb_tile(sgw_ctx* c, int precision, int system, int q, int shape) {
  if (!c) return SGW_EINVAL;
  auto set = [&](auto& S) -> int {
    using T = std::remove_reference_t<decltype(*S.r)>;
    if (q < 1 || q > c->P || q > k::cheb_max_q<T>(S.max_block_rows, shape) ||
        k::cheb_lds_bytes<T>(S.max_block_rows, q, shape) > 150 * 1024) {
      c->err = "Chebyshev tile not feasible for this system";
      return SGW_EINVAL;
    }
    S.cq = q;
    S.cshape = shape;
    return 0;
  };
  if (system != 0 && system != 1) {
    c->err = "system must be 0 (Dirichlet) or 1 (Neumann)";
    return SGW_EINVAL;
  }
  if (precision == SGW_FP64) return system == 0 ? set(c->d64.D) : set(c->d64.N);
  if (precision == SGW_FP32_IR64 && c->f32.ready)
    return system == 0 ? set(c->f32.D) : set(c->f32.N);
  c->err = "no such precision in this context";
  return SGW_EINVAL;
}

int sgw_destroy(sgw_ctx* c) {
  if (!c) return 0;
  (void)hipDeviceSynchronize();
  prof_harvest(c);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  for (void* p : c->mem) {
    if (c->has_al) c->al.free(p, c->al.user);
    else (void)hipFree(p);
  }
  if (c->hflags) (void)hipHostFree(c->hflags);
  if (c->hosc) (void)hipHostFree(c->hosc);
  if (c->hpart) (void)hipHostFree(c->hpart);
  if (c->acct_h) (void)hipHostFree(c->acct_h);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return 0;
}

int sgw_create(const sgw_problem_desc* d, const sgw_allocator* al, sgw_ctx** out) {
  if (!d || !out) return SGW_EINVAL;
  *out = nullptr;
  sgw_ctx* c = new sgw_ctx();
  if (al && al->alloc && al->free) {
    c->al = *al;
    c->has_al = true;
  }
  sgw_problem_desc dd = *d;
  if (dd.zeta == 0.0) dd.zeta = 0.25;
  if (dd.gamma == 0.0) dd.gamma = 0.5;
  if (dd.max_iter <= 0) dd.max_iter = 1000;
  if (dd.inner_max_iter <= 0) dd.inner_max_iter = 1000;
  if (!(dd.rtol > 0)) dd.rtol = 1e-8;
  if (!(dd.inner_rtol > 0)) dd.inner_rtol = 1e-3 * dd.rtol;
  if (!(dd.precond_rtol > 0)) dd.precond_rtol = dd.inner_rtol;
  if (dd.cheb_degree <= 0) dd.cheb_degree = 4;
  if (dd.L == 0) dd.p_in = dd.p_out = 0;  // deterministic medium: one mode, P = 1
  if (!(dd.ir_outer_rtol > 0)) dd.ir_outer_rtol = kIrOuterRtol;
  if (!(dd.ir_inner_rtol > 0)) dd.ir_inner_rtol = kIrInnerRtol;
  if (!(dd.ir_precond_rtol > 0)) dd.ir_precond_rtol = kIrPrecondRtol;
  if ((dd.inner_prec != SGW_INNER_CHOLESKY && dd.inner_prec != SGW_INNER_CHEBYSHEV) ||
      dd.cheb_degree > 64 || (dd.precision != SGW_FP64 && dd.precision != SGW_FP32_IR64)) {
    c->err = "inner_prec, cheb_degree or precision out of range";
    *out = c;
    return SGW_EINVAL;
  }
  c->inner_prec = dd.inner_prec;
  c->cheb_deg = dd.cheb_degree;
  c->use_graphs = dd.graphs != 0;
  int rc = build_host(dd, c->h, c->err);  // host-side validation and set-up
  if (rc) {
    *out = c;
    return rc;
  }
  if (hipGetDevice(&c->dev) != hipSuccess) {
    c->err = "no HIP device";
    *out = c;
    return SGW_EHIP;
  }
  Host& h = c->h;
  c->P = h.g.P;
  c->nk = h.g.nk;
  c->NF = h.NF;
  c->nI = h.nI;
  c->nG = h.nG;
  c->nC = h.nC;
  c->NT = h.NT;
  c->nsub = h.nsub;
  c->nn = h.nn;
  const int P = c->P;
  int GS = (P + ((P + 47) / 48) - 1) / ((P + 47) / 48);
  build_gtab(c, 8, GS);
  auto fbytes = [](const Factor& f) {
    return 8.0 * (f.lr_val.size() + f.lc_val.size() + f.dinv.size() + f.dinvT.size()) +
           4.0 * (f.lr_col.size() + f.lc_row.size() + f.lr_ptr.size() + f.lc_ptr.size());
  };
  c->factor_bytes_D = fbytes(h.fD);
  c->factor_bytes_N = fbytes(h.fN);
  // the exact triangular solves hold one nested-dissection level per workgroup
  if (dd.inner_prec == SGW_INNER_CHOLESKY &&
      (h.fD.max_level_rows > 2048 || h.fN.max_level_rows > 2048)) {
    c->err = "a nested-dissection level holds more than 2048 rows (exact subdomain preconditioner)";
    *out = c;
    return SGW_EINVAL;
  }
  c->hal_G0 = build_halo(c, h.glob, 0);
  c->hal_GI = build_halo(c, h.glob, h.nI);
  c->hal_D = build_halo(c, h.dir, 0, &h.Ioff);
  c->hal_N = build_halo(c, h.neu, 0, &h.Toff);
  for (int w = 0; w < 2; ++w)
    c->k1_generated[w] = k::sg_apply_generated(h.d.L, h.d.p_in, h.d.p_out, w ? 8 : 4);
  c->pqg = dalloc<double>(c, (size_t)std::max({P, c->k1_generated[0], c->k1_generated[1]}) *
                                 std::max(c->hal_D.ng, c->hal_N.ng));
  if (k::sg_apply_prepare() != 0) {
    c->err = "hipFuncSetAttribute failed for the SG-apply kernels";
    *out = c;
    return SGW_EHIP;
  }
  setup_prec<double>(c, c->d64, false);
  if (dd.precision == SGW_FP32_IR64) setup_prec<float>(c, c->f32, true);
  if (c->inner_prec == SGW_INNER_CHEBYSHEV) {
    if (std::max(c->d64.D.max_block_rows, c->d64.N.max_block_rows) > 4096) {
      c->err = "a subdomain block has more than 4096 rows (Chebyshev preconditioner limit)";
      *out = c;
      return SGW_EINVAL;
    }
    if (k::cheb_prepare() != 0) {
      c->err = "hipFuncSetAttribute failed for the Chebyshev kernels";
      *out = c;
      return SGW_EHIP;
    }
  }
  {
    size_t nv = (size_t)P * h.NF;
    for (double** v : {&c->U, &c->V, &c->A, &c->Um, &c->Uc, &c->Wm, &c->F})
      *v = dalloc<double>(c, nv);
    if (carry_images(h.d))
      for (double** v : {&c->GU, &c->GV, &c->GA}) *v = dalloc<double>(c, nv);
    c->hist = dalloc<double>(c, (size_t)4 * P * h.nG);
    c->gnew = dalloc<double>(c, (size_t)P * h.nG);
    c->smax = dalloc<double>(c, (size_t)P);
    c->mx = dalloc<float>(c, (size_t)P * 4 * h.nG);
    c->my = dalloc<float>(c, (size_t)P * h.nG);
  }
  c->meshbuf = dalloc<double>(c, (size_t)std::max(P, 2) * h.nn);
  c->meshbuf2 = dalloc<double>(c, (size_t)P * h.nn);
  int nbmax = std::max(64, h.nsub);  // also the row chunks of the whole-array dots (<= 64)
  c->part = dalloc<double>(c, (size_t)nbmax * P);
  c->part2 = dalloc<double>(c, (size_t)nbmax * P);
  c->ngchunk = std::max(1, std::min(16, (h.nG + 255) / 256));
  c->osc = dalloc<double>(c, (size_t)2 * c->ngchunk * P + 8);
  c->sc = dalloc<double>(c, (size_t)nbmax * 8);
  c->flags = dalloc<int>(c, 4);
  {  // row chunks of the interface part (one workgroup per chunk and mode)
    std::vector<int> gc(c->ngchunk + 1);
    for (int i = 0; i <= c->ngchunk; ++i) gc[i] = (int)((long long)h.nG * i / c->ngchunk);
    c->goff = upload(c, gc);
  }
  c->alloff = upload(c, std::vector<int>{0, h.NF});
  {  // about 64 row chunks (one workgroup per chunk and mode in a dot product)
    const int nch = std::max(1, std::min(64, (h.NF + 1023) / 1024));
    std::vector<int> fc(nch + 1);
    for (int i = 0; i <= nch; ++i) fc[i] = (int)((long long)h.NF * i / nch);
    c->fchunk = upload(c, fc);
    c->nfchunk = nch;
  }
  c->dd2mesh = upload(c, h.dd2mesh);
  std::vector<double> md(h.NF);
  for (int r = 0; r < h.NF; ++r) md[r] = h.glob.mval[r];  // slot 0 = diagonal
  c->mdiag = upload(c, md);
  c->torn_gidx = upload(c, h.torn_gidx);
  c->torn_w = upload(c, h.torn_w);
  c->gam_ptr = upload(c, h.gam_ptr);
  c->gam_torn = upload(c, h.gam_torn);
  c->gam_w = upload(c, h.gam_w);
  c->g2c = upload(c, h.g2c.empty() ? std::vector<int>{-1} : h.g2c);
  // coarse structures
  k::DCoarse& co = c->co;
  co.nC = h.nC;
  co.P = P;
  co.nk = c->nk;
  for (int s = 0; s < h.nsub; ++s) c->maxc = std::max(c->maxc, h.sc_ptr[s + 1] - h.sc_ptr[s]);
  co.maxc = c->maxc;
  if ((long long)c->maxc * P > SGW_MAX_COARSE_LOCAL) {
    c->err = "too many coarse unknowns per subdomain (corners x P above 4096)";
    *out = c;
    return SGW_EINVAL;
  }
  std::vector<std::vector<int>> cl(h.nC);
  for (size_t lc = 0; lc < h.sc_coarse.size(); ++lc) cl[h.sc_coarse[lc]].push_back((int)lc);
  std::vector<int> c_ptr{0}, c_lc;
  for (auto& v : cl) {
    c_lc.insert(c_lc.end(), v.begin(), v.end());
    c_ptr.push_back((int)c_lc.size());
  }
  co.c_ptr = upload(c, c_ptr);
  co.c_lc = upload(c, c_lc);
  co.sc_gidx = upload(c, h.sc_gidx);
  co.sc_coarse = upload(c, h.sc_coarse);
  co.sc_w = upload(c, h.sc_w);
  co.sc_ptr = upload(c, h.sc_ptr);
  co.cc_ptr = upload(c, h.cc_ptr);
  co.cc_torn = upload(c, h.cc_torn);
  co.cc_val = upload(c, h.cc_val);
  {
    std::vector<std::vector<int>> byi(P);
    for (size_t e = 0; e < h.g.v.size(); ++e) byi[h.g.i[e]].push_back((int)e);
    std::vector<int> gp{0}, gk, gj;
    std::vector<double> gv;
    for (int i = 0; i < P; ++i) {
      for (int e : byi[i]) {
        gk.push_back(h.g.k[e]);
        gj.push_back(h.g.j[e]);
        gv.push_back(h.g.v[e]);
      }
      gp.push_back((int)gk.size());
    }
    co.gi_ptr = upload(c, gp);
    co.gi_k = upload(c, gk);
    co.gi_j = upload(c, gj);
    co.gi_v = upload(c, gv);
  }
  c->rem_off_h.assign(1, 0);
  c->phi_off_h.assign(1, 0);
  c->phih_off_h.assign(1, 0);
  for (int s = 0; s < h.nsub; ++s) {
    for (int t = h.Toff[s]; t < h.Toff[s + 1]; ++t)
      if (h.torn_gidx[t] >= 0) c->rem_list_h.push_back(t);
    c->rem_off_h.push_back((int)c->rem_list_h.size());
    long long nrem = c->rem_off_h[s + 1] - c->rem_off_h[s];
    int ncs = h.sc_ptr[s + 1] - h.sc_ptr[s];
    c->phi_off_h.push_back(c->phi_off_h.back() + (long long)P * ncs * P * nrem);
    // the FP16 copy pads each row of outputs to a multiple of 4 (8-byte loads)
    c->phih_off_h.push_back(c->phih_off_h.back() + (long long)P * ncs * ((P * nrem + 3) / 4 * 4));
  }
  co.rem_off = upload(c, c->rem_off_h);
  co.rem_list = upload(c, c->rem_list_h.empty() ? std::vector<int>{0} : c->rem_list_h);
  co.phi_off = upload(c, c->phi_off_h);
  c->phi = dalloc<double>(c, (size_t)std::max<long long>(1, c->phi_off_h.back()));
  co.phi = c->phi;
  if (dd.precision == SGW_FP32_IR64) {
    c->phih = dalloc<unsigned short>(c, (size_t)std::max<long long>(4, c->phih_off_h.back()));
    co.phih = c->phih;
    co.phih_off = upload(c, c->phih_off_h);
  }
  co.max_rem = 0;
  for (int s = 0; s < h.nsub; ++s)
    co.max_rem = std::max(co.max_rem, c->rem_off_h[s + 1] - c->rem_off_h[s]);
  c->dc = dalloc<double>(c, (size_t)std::max(1, h.nC * P));
  c->uc = dalloc<double>(c, (size_t)std::max(1, h.nC * P));
  c->acct = dalloc<unsigned long long>(c, 4);
  if (hipHostMalloc((void**)&c->acct_h, 4 * sizeof(unsigned long long)) != hipSuccess)
    c->acct_h = nullptr;
  if (!c->acct_h) c->acct = nullptr;
  if (hipHostMalloc((void**)&c->hflags, 16 * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&c->hosc, (2 * (size_t)c->ngchunk * P + 8) * sizeof(double)) !=
          hipSuccess ||
      hipHostMalloc((void**)&c->hpart, 2 * (size_t)c->nfchunk * P * sizeof(double)) !=
          hipSuccess) {
    c->err = "pinned allocation failed";
    *out = c;
    return SGW_ENOMEM;
  }
  for (void* p : c->mem)
    if (!p) {
      c->err = "device allocation failed";
      *out = c;
      return SGW_ENOMEM;
    }
  if (!check_pointers(c)) {
    *out = c;
    return SGW_ENOMEM;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    c->err = "device error during upload";
    *out = c;
    return SGW_EHIP;
  }
  *out = c;
  return 0;
}

int sgw_factor(sgw_ctx* c, void* stream) {
  if (!c) return SGW_EINVAL;
  if (c->factored) {
    c->err = "the coarse grid is already factored";
    return SGW_ESTATE;
  }
  hipStream_t st = (hipStream_t)stream;
  const Host& h = c->h;
  const int P = c->P, NT = c->NT;
  if (c->nC > 0) {
    const int MP = c->maxc * P;
    c->fs = dalloc<double>(c, (size_t)c->nsub * MP * MP);
    if (!c->fs) {
      c->err = "device allocation failed (coarse set-up)";
      return SGW_ENOMEM;
    }
    HIPCHK(hipMemsetAsync(c->fs, 0, (size_t)c->nsub * MP * MP * sizeof(double), st));
    const double tol = std::min(1e-12, c->h.d.inner_rtol);
    // SGW_PROGRESS=1 reports the stages of this (long, at large P) set-up
    const char* pe = getenv("SGW_PROGRESS");
    const bool progress = pe && pe[0] == '1';
    auto t0 = std::chrono::steady_clock::now();
    auto secs = [&] {
      return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    for (int lcl = 0; lcl < c->maxc; ++lcl) {
      for (int m = 0; m < P; ++m) {
        k::fill2d<double>(P, NT, c->d64.Tt, NT, 0.0, st);
        k_basis_rhs<<<c->nsub, 256, 0, st>>>(c->co, lcl, m, c->d64.Tt, NT);
        int rc = inner_solve<double>(c, c->d64.N, true, c->d64.Tt, NT, c->d64.Yt, NT, tol,
                                     c->h.d.inner_max_iter, kSiteNeumann, st);
        if (rc < 0) return rc;
        k_basis_store<<<c->nsub, 256, 0, st>>>(c->co, lcl, m, c->d64.Yt, NT, c->fs);
      }
      if (progress)
        fprintf(stderr, "[sgw] coarse basis: corner slot %d of %d done (%.1f s)\n", lcl + 1,
                c->maxc, secs());
    }
    std::vector<double> fs((size_t)c->nsub * MP * MP);
    HIPCHK(hipMemcpyAsync(fs.data(), c->fs, fs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // coarse unknowns in corner rows (mesh rows of the corners; corners are
    // numbered in mesh order), inside a row corner by corner with the P
    // modes of a corner contiguous: F_cc is block tridiagonal over the rows
    const int nC = c->nC, n1 = h.n + 1;
    std::vector<int> crow(nC), cpos(nC);
    CoarseBlocks B;
    B.off.assign(1, 0);
    for (int ci = 0, r = -1, last = -1; ci < nC; ++ci) {
      const int yrow = h.dd2mesh[h.nI + h.c2g[ci]] / n1;
      if (yrow != last) {
        if (r >= 0) B.off.push_back(B.off.back() + cpos[ci - 1] * P + P);
        ++r;
        last = yrow;
        cpos[ci] = 0;
      } else {
        cpos[ci] = cpos[ci - 1] + 1;
      }
      crow[ci] = r;
      B.R = r + 1;
    }
    B.off.push_back(B.off.back() + cpos[nC - 1] * P + P);
    auto rows_of = [&](int r) { return B.off[r + 1] - B.off[r]; };
    B.diag.resize(B.R);
    B.sub.resize(B.R - 1);
    for (int r = 0; r < B.R; ++r) {
      B.diag[r].assign((size_t)rows_of(r) * rows_of(r), 0.0);
      if (r + 1 < B.R) B.sub[r].assign((size_t)rows_of(r + 1) * rows_of(r), 0.0);
    }
    // Galerkin entries by (i, j) for the corner self terms K~^s_cc
    std::vector<std::vector<int>> byij((size_t)P * P);
    for (size_t e = 0; e < h.g.v.size(); ++e) byij[(size_t)h.g.i[e] * P + h.g.j[e]].push_back((int)e);
    for (int sd = 0; sd < c->nsub; ++sd) {
      int lc0 = h.sc_ptr[sd], ncs = h.sc_ptr[sd + 1] - lc0;
      const double* Fs = &fs[(size_t)sd * MP * MP];
      for (int l2 = 0; l2 < ncs; ++l2)
        for (int m2 = 0; m2 < P; ++m2)
          for (int l1 = 0; l1 < ncs; ++l1)
            for (int m1 = 0; m1 < P; ++m1) {
              double v = Fs[(size_t)(m2 * c->maxc + l2) * MP + (m1 * c->maxc + l1)];
              if (l2 == l1)  // K~^s_cc: corners couple only to themselves
                for (int e : byij[(size_t)m2 * P + m1])
                  v += h.g.v[e] * h.cself[(size_t)(lc0 + l2) * c->nk + h.g.k[e]];
              const int ca = h.sc_coarse[lc0 + l2], cb = h.sc_coarse[lc0 + l1];
              const int ra = crow[ca], rb = crow[cb];
              const int wa = cpos[ca] * P + m2, wb = cpos[cb] * P + m1;
              if (ra == rb) {
                B.diag[ra][(size_t)wa * rows_of(ra) + wb] += v;
              } else if (ra == rb + 1) {  // (F + F^T) / 2 of the sub-diagonal block
                B.sub[rb][(size_t)wa * rows_of(rb) + wb] += 0.5 * v;
              } else if (rb == ra + 1) {
                B.sub[ra][(size_t)wb * rows_of(ra) + wa] += 0.5 * v;
              } else {
                c->err = "coarse couplings span more than one corner row (not a rectilinear partition)";
                return SGW_EINVAL;
              }
            }
    }
    for (int r = 0; r < B.R; ++r) {
      const int m = rows_of(r);
      std::vector<double>& D = B.diag[r];
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < i; ++j) {
          const double a = 0.5 * (D[(size_t)i * m + j] + D[(size_t)j * m + i]);
          D[(size_t)i * m + j] = a;
          D[(size_t)j * m + i] = a;
        }
    }
    std::vector<double>().swap(fs);
    CoarseFactor CF;
    const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (!coarse_factor(B, CF, threads, c->err)) return SGW_ENOTSPD;
    if (progress)
      fprintf(stderr, "[sgw] coarse factor: %d corner rows, %d unknowns (%.1f s)\n", CF.R,
              nC * P, secs());
    k::DCoarseFactor& df = c->cf;
    df.R = CF.R;
    df.n = nC * P;
    df.off = CF.off;
    auto transpose = [](const std::vector<double>& a, int nr, int nc) {
      std::vector<double> t(a.size());
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) t[(size_t)j * nr + i] = a[(size_t)i * nc + j];
      return t;
    };
    // the FP32 solver's coarse solves read FP32 copies (a preconditioner:
    // its Neumann solves stop far above FP32 rounding)
    const bool single = c->h.d.precision == SGW_FP32_IR64;
    auto to_f = [](const std::vector<double>& a) { return std::vector<float>(a.begin(), a.end()); };
    for (int r = 0; r < CF.R; ++r) {
      const int m = rows_of(r);
      const std::vector<double> lt = transpose(CF.linv[r], m, m);
      df.linv.push_back(upload(c, CF.linv[r]));
      df.linvT.push_back(upload(c, lt));
      if (single) {
        df.linvf.push_back(upload(c, to_f(CF.linv[r])));
        df.linvTf.push_back(upload(c, to_f(lt)));
      }
      if (r + 1 < CF.R) {
        const std::vector<double> bt = transpose(CF.b[r], rows_of(r + 1), m);
        df.b.push_back(upload(c, CF.b[r]));
        df.bT.push_back(upload(c, bt));
        if (single) {
          df.bf.push_back(upload(c, to_f(CF.b[r])));
          df.bTf.push_back(upload(c, to_f(bt)));
        }
      }
    }
    std::vector<int> perm(df.n);
    for (int ci = 0; ci < nC; ++ci)
      for (int m = 0; m < P; ++m) perm[B.off[crow[ci]] + cpos[ci] * P + m] = m * nC + ci;
    df.perm = upload(c, perm);
    df.wd = dalloc<double>(c, df.n);
    df.wy = dalloc<double>(c, df.n);
    df.wt = dalloc<double>(c, df.n);
    df.wx = dalloc<double>(c, df.n);
    bool ok = df.perm && df.wd && df.wy && df.wt && df.wx;
    for (auto* v : {&df.linv, &df.linvT, &df.b, &df.bT})
      for (const double* p : *v) ok = ok && p;
    for (auto* v : {&df.linvf, &df.linvTf, &df.bf, &df.bTf})
      for (const float* p : *v) ok = ok && p;
    if (!ok) {
      c->err = "device allocation failed (coarse factor)";
      return SGW_ENOMEM;
    }
    if (c->phih) {  // the FP32 solver's FP16 copy of the coarse basis
      std::vector<int> nq(c->nsub);
      std::vector<long long> nout(c->nsub);
      for (int s = 0; s < c->nsub; ++s) {
        nq[s] = P * (h.sc_ptr[s + 1] - h.sc_ptr[s]);
        nout[s] = (long long)P * (c->rem_off_h[s + 1] - c->rem_off_h[s]);
      }
      const int* dnq = upload(c, nq);
      const long long* dno = upload(c, nout);
      if (!dnq || !dno) {
        c->err = "device allocation failed (coarse basis copy)";
        return SGW_ENOMEM;
      }
      k::coarse_basis_to_half(c->co, c->nsub, dnq, dno, st);
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  c->factored = true;
  return 0;
}

// ---------------------------------------------------------------------------
// H3 (learned): per PCE mode j and interface node i, the network sees the
// deviations c_m = u_m - g_m of the last four converged interface values
// from the Newmark extrapolations made at those steps, scaled by
// s_j = max_i |c_n^j(i)|, and returns the next deviation in that scale.
// ---------------------------------------------------------------------------
// slot[j][i] = u[j][i] - g[j][i]
__global__ void k_hist_push(int P, int nG, const double* u, int ldu, const double* g,
                            double* slot) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)P * nG) return;
  const int j = (int)(q / nG), i = (int)(q % nG);
  slot[q] = u[(size_t)j * ldu + i] - g[q];
}
// s_j = max_i |slot[j][i]| (+ the smallest normal number), one workgroup per mode
__global__ __launch_bounds__(256) void k_mode_scale(int nG, const double* slot, double* smax) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double m = 0.0;
  for (int i = threadIdx.x; i < nG; i += 256) m = fmax(m, fabs(slot[(size_t)j * nG + i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) smax[j] = sh[0] + 2.2250738585072014e-308;
}
// row (j nG + i) of x: hist[slot h][j][i] / s_j, h = 0..3 oldest first
__global__ void k_guess_input(int P, int nG, const double* hist, int h0, const double* smax,
                              float* x) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)P * 4 * nG) return;
  const long long row = q >> 2;
  const int h = (int)(q & 3);
  const int j = (int)(row / nG), i = (int)(row % nG);
  const int slot = (h0 + h) & 3;
  x[q] = (float)(hist[((size_t)slot * P + j) * nG + i] / smax[j]);
}
// t[j][i] = (u_new[j][i] - g[j][i]) / s_j
__global__ void k_guess_target(int P, int nG, const double* un, int ldu, const double* g,
                               const double* smax, float* t) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)P * nG) return;
  const int j = (int)(q / nG), i = (int)(q % nG);
  t[q] = (float)((un[(size_t)j * ldu + i] - g[q]) / smax[j]);
}
// x = g + s_j y, or g where that is not finite
__global__ void k_guess_apply(int P, int nG, const double* g, const double* smax, const float* y,
                              double* x, int ldx) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)P * nG) return;
  const int j = (int)(q / nG), i = (int)(q % nG);
  const double v = g[q] + smax[j] * (double)y[q];
  x[(size_t)j * ldx + i] = isfinite(v) ? v : g[q];
}

static int grid1(long long n) { return (int)((n + 255) / 256); }

// Appends the deviation of the new interface solution (the interface part
// of u, ld NF) from this step's Newmark guess g to the history ring.
static void hist_push(sgw_ctx* c, const double* u, const double* g, hipStream_t st) {
  const int P = c->P, nG = c->nG;
  k_hist_push<<<grid1((long long)P * nG), 256, 0, st>>>(P, nG, u + c->nI, c->NF, g,
                                                       c->hist + (size_t)c->hist_pos * P * nG);
  c->hist_pos = (c->hist_pos + 1) & 3;
  c->hist_n = std::min(c->hist_n + 1, 4);
}
// network input of the current history (needs 4 entries) into c->mx
static void guess_input(sgw_ctx* c, hipStream_t st) {
  const int P = c->P, nG = c->nG;
  const int newest = (c->hist_pos + 3) & 3;
  k_mode_scale<<<P, 256, 0, st>>>(nG, c->hist + (size_t)newest * P * nG, c->smax);
  k_guess_input<<<grid1((long long)P * 4 * nG), 256, 0, st>>>(P, nG, c->hist, c->hist_pos,
                                                             c->smax, c->mx);
}

int sgw_set_state(sgw_ctx* c, const double* U, const double* V, const double* A, int where,
                  int step, void* stream) {
  if (!c) return SGW_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Host& h = c->h;
  const int P = c->P, NF = c->NF;
  const sgw_problem_desc& d = h.d;
  if (U) {
    to_dd(c, U, where, c->U, st);
  } else {
    std::vector<double> u0((size_t)P * c->nn, 0.0);
    for (int v = 0; v < c->nn; ++v) {
      double x = (v % (h.n + 1)) / (double)h.n, y = (v / (h.n + 1)) / (double)h.n;
      double r2 = (x - d.x0) * (x - d.x0) + (y - d.y0) * (y - d.y0);
      u0[v] = d.amp * std::exp(-r2 / (d.width * d.width));
    }
    HIPCHK(hipMemcpyAsync(c->meshbuf2, u0.data(), u0.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
    to_dd(c, c->meshbuf2, SGW_DEVICE, c->U, st);
    HIPCHK(hipStreamSynchronize(st));
  }
  if (V) to_dd(c, V, where, c->V, st);
  else k::fill2d<double>(P, NF, c->V, NF, 0.0, st);
  if (A) {
    to_dd(c, A, where, c->A, st);
  } else {
    // (I(x)M) A = -(K U + C V); K = (K~ - a_m I(x)M)/s_k, C = a0 I(x)M + a1 K
    const double s = h.s_k, am = h.a_m, a0 = d.alpha0, a1 = d.alpha1;
    k::axpby2d<double>(P, NF, 1.0, c->U, NF, a1, c->V, NF, c->Wm, NF, st);
    k::sg_apply<double>(c->d64.G, c->gt, &c->hal_G0, 0, NF, c->Wm, NF, c->F, NF, -1.0 / s, 0.0, 1, 0,
                        0, st);
    k::mass_apply<double>(c->d64.G, 0, NF, P, c->Wm, NF, c->F, NF, am / s, 1.0, st);
    k::mass_apply<double>(c->d64.G, 0, NF, P, c->V, NF, c->F, NF, -a0, 1.0, st);
    int rc = mass_solve(c, c->F, c->A, st);
    if (rc) return rc;
  }
  c->g_valid = false;  // K~ of the new state not formed yet
  // the learned guess starts a new history with this state
  c->hist_n = 0;
  c->hist_pos = 0;
  HIPCHK(hipStreamSynchronize(st));
  c->stepno = step;
  c->has_state = true;
  return 0;
}

int sgw_get_state(sgw_ctx* c, double* U, double* V, double* A, int where, void* stream) {
  if (!c) return SGW_EINVAL;
  if (!c->has_state) {
    c->err = "no state";
    return SGW_ESTATE;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (U && (rc = from_dd(c, c->U, U, where, st))) return rc;
  if (V && (rc = from_dd(c, c->V, V, where, st))) return rc;
  if (A && (rc = from_dd(c, c->A, A, where, st))) return rc;
  return 0;
}

int sgw_step(sgw_ctx* c, int nsteps, void* stream, sgw_step_stats* stats) {
  if (!c) return SGW_EINVAL;
  if (!c->factored || !c->has_state) {
    c->err = "sgw_step needs sgw_factor and sgw_set_state first";
    return SGW_ESTATE;
  }
  hipStream_t st = (hipStream_t)stream;
  const Host& h = c->h;
  const sgw_problem_desc& d = h.d;
  const int P = c->P, NF = c->NF, nI = c->nI, nG = c->nG;
  sgw_step_stats s{};
  c->inner_its = 0;
  c->inner_solves = 0;
  int warn = 0;
  for (int n = 0; n < nsteps; ++n) {
    // H1: predictor and effective force F~ = M (Um + wc Uc) + (a1/s) K~ Uc
    const double wc = d.alpha0 - d.alpha1 * h.a_m / h.s_k;
    const bool images = carry_images(d);
    if (images) {
      if (!c->g_valid) {  // first step from this state: K~ U, K~ V, K~ A
        K1<double>(c, c->d64.G, &c->hal_G0, 0, NF, c->U, NF, c->GU, NF, 1.0, 0.0, st);
        K1<double>(c, c->d64.G, &c->hal_G0, 0, NF, c->V, NF, c->GV, NF, 1.0, 0.0, st);
        K1<double>(c, c->d64.G, &c->hal_G0, 0, NF, c->A, NF, c->GA, NF, 1.0, 0.0, st);
        c->g_valid = true;
      }
      k::newmark_predict_g(P, NF, c->U, c->V, c->A, c->GU, c->GV, c->GA, d.dt, d.zeta, d.gamma,
                           wc, d.alpha1 / h.s_k, c->Um, c->Wm, c->F, st);
      k::mass_apply<double>(c->d64.G, 0, NF, P, c->Wm, NF, c->F, NF, 1.0, 1.0, st);
    } else {
      k::newmark_predict(P, NF, NF, c->U, c->V, c->A, d.dt, d.zeta, d.gamma, wc, c->Um, c->Uc,
                         c->Wm, st);
      k::mass_apply<double>(c->d64.G, 0, NF, P, c->Wm, NF, c->F, NF, 1.0, 0.0, st);
      if (d.alpha1 != 0.0)
        K1<double>(c, c->d64.G, &c->hal_G0, 0, NF, c->Uc, NF, c->F, NF, d.alpha1 / h.s_k, 1.0,
                   st);
    }
    // H3: initial interface guess.  Newmark extrapolation g = U + dt V +
    // dt^2/2 A on the interface (also the reference of the learned
    // correction); the previous solution; or g plus the network's correction
    // (with fewer than 4 past steps or no model attached: g)
    const bool learned = d.guess == SGW_GUESS_LEARNED && c->mlp && c->hist_n >= 4;
    const long long rows = (long long)P * nG;  // network rows of a step
    const bool recording = c->rec_x && c->hist_n >= 4 && c->rec_n + rows <= c->rec_cap;
    k::axpby2d<double>(P, nG, 1.0, c->U + nI, NF, d.dt, c->V + nI, NF, c->gnew, nG, st);
    k::axpby2d<double>(P, nG, 1.0, c->gnew, nG, 0.5 * d.dt * d.dt, c->A + nI, NF, c->gnew, nG,
                       st);
    if (learned || recording) guess_input(c, st);
    if (learned) {
      int mrc = sgw::mlp_forward(c->mlp, c->mx, c->my, (int)rows, st);
      if (mrc < 0) {
        c->err = "learned guess: " + c->mlp->err;
        return mrc;
      }
      k_guess_apply<<<grid1((long long)P * nG), 256, 0, st>>>(P, nG, c->gnew, c->smax, c->my,
                                                             c->d64.X + nI, NF);
    } else if (d.guess == SGW_GUESS_PREV) {
      k::copy2d<double, double>(P, nG, c->U + nI, NF, c->d64.X + nI, NF, 1.0, st);
    } else {
      k::copy2d<double, double>(P, nG, c->gnew, nG, c->d64.X + nI, NF, 1.0, st);
    }
    const double* fallback = learned ? c->gnew : nullptr;
    int its = 0, sweeps = 0;
    double rel = 0.0;
    int rc;
    if (d.precision == SGW_FP32_IR64) {
      // the refinement starts from the whole previous (or extrapolated) state
      k::copy2d<double, double>(P, nI, c->U, NF, c->d64.X, NF, 1.0, st);
      if (d.guess != SGW_GUESS_PREV) {
        k::axpby2d<double>(P, nI, 1.0, c->U, NF, d.dt, c->V, NF, c->d64.X, NF, st);
        k::axpby2d<double>(P, nI, 1.0, c->d64.X, NF, 0.5 * d.dt * d.dt, c->A, NF, c->d64.X, NF, st);
      }
      // X = U + cv V + ca A everywhere unless the learned correction moved
      // the interface: then the first residual needs the apply
      const double x0[2] = {d.guess == SGW_GUESS_PREV ? 0.0 : d.dt,
                            d.guess == SGW_GUESS_PREV ? 0.0 : 0.5 * d.dt * d.dt};
      rc = ir_solve(c, c->F, c->d64.X, st, its, sweeps, rel, fallback,
                    images && !learned ? x0 : nullptr);
      s.ir_sweeps += sweeps;
    } else {
      Tols tl{d.rtol, d.inner_rtol, d.precond_rtol, d.max_iter, d.inner_max_iter};
      rc = dd_solve<double>(c, c->d64, tl, c->F, c->d64.X, st, its, rel, fallback);
    }
    if (rc < 0) {
      c->g_valid = false;
      return rc;
    }
    warn |= rc;
    // H11: training sample (history, correction of the Newmark guess), then
    // the new solution joins the history
    if (recording) {
      HIPCHK(hipMemcpyAsync(c->rec_x + (size_t)c->rec_n * 4, c->mx,
                            (size_t)rows * 4 * sizeof(float), hipMemcpyDeviceToDevice, st));
      k_guess_target<<<grid1(rows), 256, 0, st>>>(P, nG, c->d64.X + nI, NF, c->gnew, c->smax,
                                                  c->rec_t + (size_t)c->rec_n);
      c->rec_n += rows;
    }
    hist_push(c, c->d64.X, c->gnew, st);
    // H6: Newmark update
    if (images)  // ir_solve leaves R = F - K~ X of the accepted X
      k::newmark_update_g(P, NF, c->d64.X, c->Um, c->F, c->d64.R, c->V, c->A, c->GU, c->GV,
                          c->GA, d.dt, d.zeta, d.gamma, st);
    else
      k::newmark_update(P, NF, NF, c->d64.X, c->Um, c->V, c->A, d.dt, d.zeta, d.gamma, st);
    std::swap(c->U, c->d64.X);
    s.steps++;
    s.outer_iters += its;
    s.outer_iters_max = std::max(s.outer_iters_max, its);
    s.last_rel_res = rel;
    c->stepno++;
  }
  HIPCHK(hipStreamSynchronize(st));
  prof_harvest(c);
  s.inner_iters = c->inner_its;
  s.inner_solves = c->inner_solves;
  if (stats) *stats = s;
  return warn ? SGW_NOT_CONVERGED : 0;
}

// H9: several independent problems in one call.  Each context advances on
// its own stream from its own host thread, so the kernels of the problems
// overlap on the GPU while every problem keeps its own convergence checks.
int sgw_step_batch(sgw_ctx** ctx, int n, int nsteps, void** streams, sgw_step_stats* stats,
                   int* status) {
  if (!ctx || n <= 0 || nsteps < 0) return SGW_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctx[i]) return SGW_EINVAL;
    for (int q = 0; q < i; ++q)
      if (ctx[q] == ctx[i]) return SGW_EINVAL;  // a context is not thread-safe
  }
  for (int i = 0; i < n; ++i)
    if (!streams && !ctx[i]->own_stream &&
        hipStreamCreateWithFlags(&ctx[i]->own_stream, hipStreamNonBlocking) != hipSuccess) {
      ctx[i]->err = "stream creation failed";
      return SGW_EHIP;
    }
  std::vector<int> rc(n, 0);
  std::vector<std::thread> th;
  th.reserve(n);
  for (int i = 0; i < n; ++i)
    th.emplace_back([&, i] {
      if (hipSetDevice(ctx[i]->dev) != hipSuccess) {
        rc[i] = SGW_EHIP;
        return;
      }
      void* st = streams ? streams[i] : (void*)ctx[i]->own_stream;
      rc[i] = sgw_step(ctx[i], nsteps, st, stats ? &stats[i] : nullptr);
    });
  for (auto& t : th) t.join();
  int worst = 0;
  for (int i = 0; i < n; ++i) {
    if (status) status[i] = rc[i];
    if (rc[i] < 0 && worst >= 0) worst = rc[i];
    if (rc[i] > 0 && worst == 0) worst = SGW_NOT_CONVERGED;
  }
  return worst;
}

int sgw_guess_train(sgw_ctx* c, const sgw_train_desc* td, void* stream, float* final_loss) {
  if (!c || !td || td->nsteps < 0 || td->epochs < 0 || (td->epochs > 0 && td->batch <= 0) ||
      (td->epochs > 0 && !(td->lr > 0)))
    return SGW_EINVAL;
  if (!c->mlp) {
    c->err = "sgw_guess_train needs a network (sgw_set_guess_model)";
    return SGW_ESTATE;
  }
  hipStream_t st = (hipStream_t)stream;
  if (td->clear) c->gs_n = 0;
  const long long rows = (long long)c->P * c->nG;
  const long long need = c->gs_n + rows * td->nsteps;
  if (need > c->gs_cap) {  // grow the store, keeping its samples
    float* nx = dalloc<float>(c, (size_t)need * 4);
    float* nt = dalloc<float>(c, (size_t)need);
    if (!nx || !nt) {
      c->err = "device allocation failed (training samples)";
      return SGW_ENOMEM;
    }
    if (c->gs_n > 0) {
      HIPCHK(hipMemcpyAsync(nx, c->gs_x, (size_t)c->gs_n * 4 * sizeof(float),
                            hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(nt, c->gs_t, (size_t)c->gs_n * sizeof(float),
                            hipMemcpyDeviceToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    dfree(c, c->gs_x);
    dfree(c, c->gs_t);
    c->gs_x = nx;
    c->gs_t = nt;
    c->gs_cap = need;
  }
  int rc = 0;
  if (td->nsteps > 0) {
    c->rec_x = c->gs_x + (size_t)c->gs_n * 4;
    c->rec_t = c->gs_t + (size_t)c->gs_n;
    c->rec_cap = c->gs_cap - c->gs_n;
    c->rec_n = 0;
    rc = sgw_step(c, td->nsteps, stream, nullptr);
    c->gs_n += c->rec_n;
    c->rec_x = c->rec_t = nullptr;
    c->rec_cap = 0;
    if (rc < 0) return rc;
  }
  if (td->epochs > 0) {
    if (c->gs_n <= 0 || c->gs_n > 0x7fffffffLL) {
      c->err = "no training samples (or more than 2^31)";
      return SGW_EINVAL;
    }
    int trc = sgw_mlp_train(c->mlp, c->gs_x, c->gs_t, (int)c->gs_n, td->epochs, td->batch,
                            td->lr, td->seed, stream, final_loss);
    if (trc < 0) {
      c->err = "training failed: " + c->mlp->err;
      return trc;
    }
  }
  return rc;
}

int sgw_read_pce(sgw_ctx* c, double* U, int where, void* stream) {
  if (!c || !U) return SGW_EINVAL;
  return sgw_get_state(c, U, nullptr, nullptr, where, stream);
}

int sgw_solve(sgw_ctx* c, const double* F, double* U, void* stream, sgw_step_stats* stats) {
  if (!c || !F || !U) return SGW_EINVAL;
  if (!c->factored) {
    c->err = "sgw_solve needs sgw_factor first";
    return SGW_ESTATE;
  }
  hipStream_t st = (hipStream_t)stream;
  c->inner_its = 0;
  c->inner_solves = 0;
  to_dd(c, F, SGW_DEVICE, c->Wm, st);
  to_dd(c, U, SGW_DEVICE, c->d64.X, st);
  int its = 0;
  double rel = 0.0;
  const sgw_problem_desc& d = c->h.d;
  Tols tl{d.rtol, d.inner_rtol, d.precond_rtol, d.max_iter, d.inner_max_iter};
  int rc = dd_solve<double>(c, c->d64, tl, c->Wm, c->d64.X, st, its, rel);
  if (rc < 0) return rc;
  int rc2 = from_dd(c, c->d64.X, U, SGW_DEVICE, st);
  if (rc2) return rc2;
  HIPCHK(hipStreamSynchronize(st));
  if (stats) {
    sgw_step_stats s{};
    s.outer_iters = its;
    s.outer_iters_max = its;
    s.inner_iters = c->inner_its;
    s.inner_solves = c->inner_solves;
    s.last_rel_res = rel;
    *stats = s;
  }
  return rc;
}

int sgw_read_moments(sgw_ctx* c, double* mean, double* var, int where, void* stream) {
  if (!c) return SGW_EINVAL;
  if (!c->has_state) {
    c->err = "no state";
    return SGW_ESTATE;
  }
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = (size_t)c->nn * sizeof(double);
  double* dm = where == SGW_HOST ? c->meshbuf : mean;
  double* dv = where == SGW_HOST ? c->meshbuf + c->nn : var;
  if (dm) HIPCHK(hipMemsetAsync(dm, 0, bytes, st));
  if (dv) HIPCHK(hipMemsetAsync(dv, 0, bytes, st));
  k_moments<<<(c->NF + 255) / 256, 256, 0, st>>>(c->P, c->NF, c->dd2mesh, c->U,
                                                 mean ? dm : nullptr, var ? dv : nullptr);
  if (where == SGW_HOST) {
    if (mean) HIPCHK(hipMemcpyAsync(mean, dm, bytes, hipMemcpyDeviceToHost, st));
    if (var) HIPCHK(hipMemcpyAsync(var, dv, bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return 0;
}

int sgw_apply_operator(sgw_ctx* c, const double* X, double* Y, int precision, void* stream) {
  if (!c || !X || !Y) return SGW_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int P = c->P, NF = c->NF;
  to_dd(c, X, SGW_DEVICE, c->Wm, st);
  if (precision == SGW_FP32_IR64) {
    if (!c->f32.ready) {
      c->err = "the FP32 operator exists only for precision SGW_FP32_IR64";
      return SGW_ESTATE;
    }
    k::copy2d<float, double>(P, NF, c->Wm, NF, c->f32.Fb, NF, 1.0, st);
    K1<float>(c, c->f32.G, &c->hal_G0, 0, NF, c->f32.Fb, NF, c->f32.Xb, NF, 1.0, 0.0, st);
    k::copy2d<double, float>(P, NF, c->f32.Xb, NF, c->F, NF, 1.0, st);
  } else {
    K1<double>(c, c->d64.G, &c->hal_G0, 0, NF, c->Wm, NF, c->F, NF, 1.0, 0.0, st);
  }
  return from_dd(c, c->F, Y, SGW_DEVICE, st);
}

}  // extern "C"

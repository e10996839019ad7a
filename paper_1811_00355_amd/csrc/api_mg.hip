// C ABI, part 2: multigrid setup (Sec. 2 adaptive setup), transfer, coarse
// operator, the even-odd coarse GMRES, the preconditioner M of Eq. (5) and the
// flexible GMRES outer solver.  Host code here only sequences kernels and
// reads per-RHS convergence flags; all arithmetic runs on the device.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <functional>
#include <cmath>
#include <cstring>
#include <map>

#include "dd_internal.h"
#include "ktimer.h"

void launch_coarse_perm(const GeomDev& g, dd_dtype vt, int nc, int nrhs, int to_packed, const void* src, void* dst,
                        hipStream_t st);

// ---------------------------------------------------------------------------
// device arena: one allocation, carved into aligned pieces
// ---------------------------------------------------------------------------
struct Arena {
  dd_ctx* ctx = nullptr;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool sizing = true;
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return sizing ? nullptr : reinterpret_cast<T*>(base + off);
  }
};

// per-RHS Hessenberg state of one GMRES(m)
struct Arnoldi {
  int m = 0;
  double2 *H, *sn, *gv, *h1, *h2, *nrm2, *y;
  double *cs, *tolabs, *beta, *est, *hnext;
  int *active, *kcyc, *finished;
  void carve(Arena& a, int nrhs, int mm) {
    m = mm;
    H = a.take<double2>((size_t)nrhs * m * (m + 1));
    sn = a.take<double2>((size_t)nrhs * m);
    gv = a.take<double2>((size_t)nrhs * (m + 1));
    h1 = a.take<double2>((size_t)nrhs * (m + 1));
    h2 = a.take<double2>((size_t)nrhs * (m + 1));
    nrm2 = a.take<double2>(nrhs);
    y = a.take<double2>((size_t)nrhs * m);
    hnext = a.take<double>(nrhs);
    cs = a.take<double>((size_t)nrhs * m);
    tolabs = a.take<double>(nrhs);
    beta = a.take<double>(nrhs);
    est = a.take<double>(nrhs);
    active = a.take<int>(nrhs);
    kcyc = a.take<int>(nrhs);
    finished = a.take<int>(nrhs);
  }
};

struct Workspace {
  int nrhs = 0;
  bool outer = false;
  Arena arena;
  // V-cycle (inner dtype)
  void *vin = nullptr, *xs = nullptr;
  // coarse vectors (inner dtype) and the coarse Krylov basis
  void *cb, *cy, *cr, *cw, *ct1, *ct2, *cres, *CV;
  void* cv32;   // FP32 copy of the current basis vector when the basis is stored in FP16
  // storage type the coarse basis CV was last written in.  The basis kernels
  // read every stored vector up to the longest cycle and weight the ones a
  // masked right-hand side never wrote by zero, so those must hold finite
  // values: FP32 words read as FP16 pairs need not be, hence CV is cleared
  // when the basis type changes.
  dd_dtype cv_type = DD_F32;
  size_t cv_bytes = 0;
  Arnoldi ca;
  // outer solver
  double2 *b64, *x64, *w64, *zt64, *V64;
  void* Z;
  Arnoldi fa;
  double* partial;
  int* citers = nullptr;   // coarse Arnoldi steps of the device-driven solves (whole-M graphs)
  double2* mr = nullptr;   // minimal-residual smoother of a third level: <Ar, r>, <Ar, Ar>, alpha per RHS
  int* hflags = nullptr;   // pinned host mirror: active[nrhs], kcyc[nrhs]
  double* hvals = nullptr; // pinned host mirror: est[nrhs], tolabs[nrhs], nrm[nrhs]
  // captured coarse GMRES chunks, keyed by (nrhs, dtype, basis dtype, block dtype, waves per workgroup,
  // half matrix cores, first iteration, length, ends cycle), i.e. every launch choice baked into a capture;
  // they hold this arena's addresses and die with it
  hipStream_t cap = nullptr;
  struct Captured {
    hipGraphExec_t exec;
    double bytes, flops;   // algorithmic work of the captured launches, added at every replay
  };
  std::map<std::array<int, 9>, Captured> graphs;
  // whole preconditioner M captured per (nrhs, launch and arithmetic choices, input and output buffers)
  std::map<std::array<long long, 12>, Captured> mgraphs;
};

static dd_dtype inner_vt(const dd_mg* mg) { return mg->p.inner_dtype == DD_F64 ? DD_F64 : DD_F32; }
static dd_dtype op_dtype(const dd_mg* mg) { return mg->p.inner_dtype == DD_F64 ? DD_F64 : mg->p.store_dtype; }
static const void* P_inner(const dd_mg* mg) { return mg->p.inner_dtype == DD_F64 ? (const void*)mg->P64 : mg->Pst; }
static dd_dtype P_inner_dt(const dd_mg* mg) { return mg->p.inner_dtype == DD_F64 ? DD_F64 : mg->vstore; }

// Sizes that fix the workspace layout (also computed without a setup, for the
// footprint query).
struct WsShape {
  long long V, Vc, Vch;
  int nc;        // coarse components per site (2n)
  int mc, m;     // coarse GMRES restart, outer FGMRES restart
  dd_dtype vt;   // inner vector dtype
};

static WsShape ws_shape(const dd_mg* mg) {
  const GeomDev& G = mg->g->geo;
  return {G.V, G.Vc, G.Vch, mg->nc, mg->p.coarse_restart, mg->p.fgmres_restart, inner_vt(mg)};
}

// fine = false: the coarse solve's part only (no fine V-cycle vectors, no
// outer solver), for the allocation-free coarse solve.
static void carve_ws(Workspace& w, const WsShape& sh, int nrhs, bool outer, bool fine_part = true) {
  Arena& a = w.arena;
  const long long V = sh.V;
  const long long fine = 12LL * V * nrhs;
  const long long coarse = sh.Vc * sh.nc * nrhs;
  const size_t vb = vector_pair_bytes(sh.vt);
  const int mc = sh.mc;
  w.vin = fine_part ? a.take<char>(fine * vb) : nullptr;
  w.xs = fine_part ? a.take<char>(fine * vb) : nullptr;
  w.cb = a.take<char>(coarse * vb);
  w.cy = a.take<char>(coarse * vb);
  w.cr = a.take<char>(coarse * vb);
  w.cw = a.take<char>(coarse * vb);
  w.ct1 = a.take<char>(coarse * vb);
  w.ct2 = a.take<char>(coarse * vb);
  w.cres = a.take<char>(coarse * vb);
  w.cv32 = a.take<char>(coarse * sizeof(float2));
  w.cv_bytes = (size_t)(mc + 1) * coarse * vb;
  w.CV = a.take<char>(w.cv_bytes);
  w.ca.carve(a, nrhs, mc);
  int nblk = fine_part ? dots_blocks(12LL * V, nrhs) : 1;
  int nblk_c = dots_blocks(sh.Vc * sh.nc, nrhs);
  if (nblk_c > nblk) nblk = nblk_c;
  size_t np = (size_t)nrhs * 16 * nblk * 2;   // launch_dots: 16 vectors per launch
  // one-pass Gram-Schmidt: nv <= restart vectors over gs_blocks(count) tiles
  size_t np_gs = (size_t)nrhs * mc * gs_blocks(sh.Vch * (long long)sh.nc) * 2;
  if (outer) {
    const size_t np_outer = (size_t)nrhs * sh.m * gs_blocks(12LL * V) * 2;
    if (np_outer > np_gs) np_gs = np_outer;
  }
  if (np_gs > np) np = np_gs;
  w.partial = a.take<double>(np);
  w.citers = a.take<int>(1);
  w.b64 = w.x64 = w.w64 = w.zt64 = w.V64 = nullptr;
  w.Z = nullptr;
  if (outer) {
    const int m = sh.m;
    w.b64 = a.take<double2>(fine);
    w.x64 = a.take<double2>(fine);
    w.w64 = a.take<double2>(fine);
    w.zt64 = a.take<double2>(fine);
    w.V64 = a.take<double2>((size_t)(m + 1) * fine);
    w.Z = a.take<char>((size_t)m * fine * vb);
    w.fa.carve(a, nrhs, m);
  }
}

// device bytes of the workspace for nrhs right-hand sides (the arena plus its alignment slack)
static size_t ws_bytes(const WsShape& sh, int nrhs, bool outer) {
  Workspace w;
  w.arena.sizing = true;
  carve_ws(w, sh, nrhs, outer);
  return w.arena.used + 256;
}

static void destroy_ws(dd_ctx* ctx, Workspace* w) {
  if (!w) return;
  dd_free(ctx, w->arena.base, w->arena.cap);
  if (w->hflags) (void)hipHostFree(w->hflags);
  if (w->hvals) (void)hipHostFree(w->hvals);
  for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  for (auto& kv : w->mgraphs) (void)hipGraphExecDestroy(kv.second.exec);
  if (w->cap) (void)hipStreamDestroy(w->cap);
  delete w;
}

static void free_ws(dd_mg* mg) {
  destroy_ws(mg->ctx, mg->ws);
  mg->ws = nullptr;
}

// A workspace for nrhs right-hand sides laid out by carve(w) (called once to
// size the arena, once to place it), zero-filled, with its pinned host mirrors.
template <typename Carve>
static dd_status alloc_ws(dd_ctx* ctx, int nrhs, Carve carve, Workspace** out) {
  Workspace* w = new Workspace();
  w->nrhs = nrhs;
  w->arena.ctx = ctx;
  w->arena.sizing = true;
  carve(*w);
  const size_t bytes = w->arena.used + 256;
  dd_status st = dd_alloc(ctx, (void**)&w->arena.base, bytes);
  if (st) {
    delete w;
    return st;
  }
  w->arena.cap = bytes;
  w->arena.sizing = false;
  // start from finite values everywhere (Krylov bases are read up to the longest cycle)
  (void)hipMemset(w->arena.base, 0, bytes);
  w->arena.used = 0;
  carve(*w);
  if (hipHostMalloc((void**)&w->hflags, sizeof(int) * 2 * nrhs) != hipSuccess ||
      hipHostMalloc((void**)&w->hvals, sizeof(double) * 3 * nrhs) != hipSuccess) {
    destroy_ws(ctx, w);
    return dd_fail(ctx, DD_ENOMEM, "pinned host buffers");
  }
  *out = w;
  return DD_OK;
}

static dd_status ensure_ws(dd_mg* mg, int nrhs, bool outer) {
  Workspace* w = mg->ws;
  if (w && w->nrhs >= nrhs && (w->outer || !outer)) return DD_OK;
  if (w) {
    if (w->nrhs > nrhs) nrhs = w->nrhs;
    outer = outer || w->outer;
    free_ws(mg);
  }
  const WsShape sh = ws_shape(mg);
  return alloc_ws(mg->ctx, nrhs,
                  [&](Workspace& x) {
                    x.outer = outer;
                    carve_ws(x, sh, nrhs, outer);
                  },
                  &mg->ws);
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
static int count_active(Workspace* w, const int* dev_active, int nrhs, hipStream_t st) {
  (void)hipMemcpyAsync(w->hflags, dev_active, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  int c = 0;
  for (int r = 0; r < nrhs; ++r) c += w->hflags[r] != 0;
  return c;
}

// longest cycle over the RHS (kcyc copied to hflags[nrhs..2 nrhs))
static int max_kcyc(Workspace* w, Arnoldi& a, int nrhs, hipStream_t st) {
  (void)hipMemcpyAsync(w->hflags + nrhs, a.kcyc, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  int k = 0;
  for (int r = 0; r < nrhs; ++r) k = w->hflags[nrhs + r] > k ? w->hflags[nrhs + r] : k;
  return k;
}

// squared norms of nrhs vectors (count entries at stride ld) into out[r].x
static void norms2(Workspace* w, dd_dtype vt, int nrhs, long long count, long long ld, const void* x, double2* out,
                   hipStream_t st) {
  int nblk = dots_blocks(count, nrhs);
  launch_dots(vt, vt, nrhs, count, ld, x, 1, 0, x, w->partial, nblk, out, 1, 0, st);
}

// classical Gram-Schmidt of w against the basis V_0..V_{nv-1}, `passes` times
// (h1, then h2), then |w|^2 -> a.nrm2.  One pass: the whole basis in two sweeps
// (dots, then axpy + norm).  Two passes with nv <= 16: dots, then (axpy +
// second dots), then (axpy + norm) -- three sweeps of V.  After one pass the
// step's Arnoldi kernel reads no second-pass coefficients (h2 = null).
static void cgs(Workspace* ws, Arnoldi& a, dd_dtype vt, int nrhs, long long count, long long ld, const void* V,
                long long vstride, int nv, void* w, int passes, hipStream_t st, dd_dtype bt) {
  // bt: dtype of the basis V (vt, or DD_F16 for an FP16 basis with FP32 vectors)
  if (passes == 1 && nv <= gs_max_nv()) {
    launch_gs_dots(bt, vt, nrhs, count, ld, V, nv, vstride, w, ws->partial, a.h1, a.m + 1, st);
    launch_gs_axpy_norm(bt, vt, nrhs, count, ld, V, nv, vstride, a.h1, a.m + 1, w, ws->partial, a.nrm2, st);
    return;
  }
  int nblk = dots_blocks(count, nrhs);
  launch_dots(bt, vt, nrhs, count, ld, V, nv, vstride, w, ws->partial, nblk, a.h1, a.m + 1, 0, st);
  if (passes == 2 && nv <= 16) {
    launch_axpy_dots(vt, nrhs, count, ld, V, nv, vstride, a.h1, a.m + 1, w, ws->partial, nblk, a.h2, a.m + 1, st, bt);
    launch_axpy_norm(vt, nrhs, count, ld, V, nv, vstride, a.h2, a.m + 1, w, ws->partial, nblk, a.nrm2, st, bt);
    return;
  }
  if (passes == 2) {
    launch_multi_axpy(bt, vt, nrhs, count, ld, V, nv, vstride, a.h1, a.m + 1, 0, -1.0, w, st);
    launch_dots(bt, vt, nrhs, count, ld, V, nv, vstride, w, ws->partial, nblk, a.h2, a.m + 1, 0, st);
    launch_multi_axpy(bt, vt, nrhs, count, ld, V, nv, vstride, a.h2, a.m + 1, 0, -1.0, w, st);
    launch_dots(vt, vt, nrhs, count, ld, w, 1, 0, w, ws->partial, nblk, a.nrm2, 1, 0, st);
    return;
  }
  launch_multi_axpy(bt, vt, nrhs, count, ld, V, nv, vstride, a.h1, a.m + 1, 0, -1.0, w, st);
  launch_dots(vt, vt, nrhs, count, ld, w, 1, 0, w, ws->partial, nblk, a.nrm2, 1, 0, st);
}

// ---------------------------------------------------------------------------
// coarse even-odd solve
// ---------------------------------------------------------------------------
struct CoarseOps {
  const GeomDev* g;
  dd_dtype vt;
  int nc;
  const void *Dc, *Dinv;
  int spw;       // FP32 coarse apply: sites per workgroup
  dd_dtype bt;   // storage of the blocks (FP32 vectors may use FP32, FP16 or BF16 blocks)
  bool hm;          // half blocks on half-precision MFMA
  dd_dtype basis;   // storage of the GMRES basis: vt, or DD_F16 with FP32 vectors
  size_t bb;        // bytes of one basis element
};

static CoarseOps coarse_ops(const dd_mg* mg, dd_dtype vt) {
  CoarseOps c;
  c.g = &mg->g->geo;
  c.vt = vt;
  c.nc = mg->nc;
  const bool half = vt == DD_F32 && mg->Dch && mg->g->tune.coarse_half;
  c.Dc = vt == DD_F64 ? (const void*)mg->Dc64 : half ? (const void*)mg->Dch : (const void*)mg->Dc32;
  c.Dinv = vt == DD_F64 ? (const void*)mg->Dinv64 : half ? (const void*)mg->Dinvh : (const void*)mg->Dinv32;
  c.bt = vt == DD_F64 ? DD_F64 : half ? mg->vstore : DD_F32;
  c.spw = mg->g->tune.coarse_spw;
  c.hm = mg->g->tune.coarse_mfma_half != 0;
  c.basis = (vt == DD_F32 && mg->g->tune.coarse_basis_half) ? DD_F16 : vt;
  c.bb = c.basis == DD_F16 ? sizeof(__half2) : vector_pair_bytes(vt);
  return c;
}

// out_e = S v_e = D_ee v_e - D_eo D_oo^-1 D_oe v_e   (t1, t2 scratch, odd parts used)
static void schur_apply(const CoarseOps& c, int nrhs, const void* v, void* out, void* t1, void* t2, hipStream_t st) {
  const GeomDev& g = *c.g;
  launch_coarse_mv(g, c.vt, c.nc, c.Dc, c.Dinv, 0, nrhs, g.Vch, g.Vch, 0.0, nullptr, 1.0, v, 0.0, nullptr, t1, st, c.spw, c.bt, c.hm);
  launch_coarse_mv(g, c.vt, c.nc, c.Dc, c.Dinv, 1, nrhs, g.Vch, g.Vch, 1.0, t1, 0.0, nullptr, 0.0, nullptr, t2, st, c.spw, c.bt, c.hm);
  launch_coarse_mv(g, c.vt, c.nc, c.Dc, c.Dinv, 0, nrhs, 0, g.Vch, 1.0, v, -1.0, t2, 0.0, nullptr, out, st, c.spw, c.bt, c.hm);
}

// Arnoldi steps j0 .. j0+len-1 of one coarse GMRES cycle: w = S v_j, Gram-Schmidt,
// Givens update, v_{j+1} = w / |w| (not after the cycle's last step).  Launches
// only, no host synchronisation, so the sequence can be captured as a graph.
static void issue_chunk(const CoarseOps& c, Workspace* w, Arnoldi& a, int passes, int nrhs, long long ce,
                        long long ld, long long vs, char* CV, int j0, int len, bool ends, hipStream_t st) {
  const bool half = c.basis == DD_F16;   // the operator then reads v_j from its FP32 copy (w->cv32)
  for (int j = j0; j < j0 + len; ++j) {
    schur_apply(c, nrhs, half ? w->cv32 : CV + (size_t)j * vs * c.bb, w->cw, w->ct1, w->ct2, st);
    cgs(w, a, c.vt, nrhs, ce, ld, CV, vs, j + 1, w->cw, passes, st, c.basis);
    launch_arnoldi(nrhs, a.m, j, a.h1, passes == 2 ? a.h2 : nullptr, a.nrm2, a.H, a.cs, a.sn, a.gv, a.tolabs,
                   a.active, a.kcyc, a.est, a.hnext, st);
    if (ends && j + 1 == j0 + len) break;
    launch_normalize(c.vt, nrhs, ce, ld, w->cw, nullptr, a.hnext, a.active, CV + (size_t)(j + 1) * vs * c.bb, st,
                     c.basis, half ? w->cv32 : nullptr);
  }
}

// Run a chunk on `st`: directly, or by replaying its graph (captured on first use
// on the workspace's own stream; capturing launches nothing).
static dd_status run_chunk(dd_ctx* ctx, int passes, Workspace* w, bool graphs, const CoarseOps& c, int nrhs,
                           long long ce, long long ld, long long vs, int j0, int len, bool ends, hipStream_t st) {
  Arnoldi& a = w->ca;
  char* CV = (char*)w->CV;
  if (!graphs) {
    issue_chunk(c, w, a, passes, nrhs, ce, ld, vs, CV, j0, len, ends, st);
    return DD_OK;
  }
  const std::array<int, 9> key = {nrhs, (int)c.vt, (int)c.basis, (int)c.bt, c.spw, c.hm ? 1 : 0, j0, len, ends ? 1 : 0};
  auto it = w->graphs.find(key);
  if (it == w->graphs.end()) {
    if (!w->cap) DD_HIP(ctx, hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking));
    DD_HIP(ctx, hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
    double b0, f0, b1, f1;
    ktimer_model(&b0, &f0);
    ktimer_suspend(true);
    issue_chunk(c, w, a, passes, nrhs, ce, ld, vs, CV, j0, len, ends, w->cap);
    ktimer_suspend(false);
    ktimer_model(&b1, &f1);
    ktimer_model_set(b0, f0);   // capturing executes nothing; the replay below accounts for it
    hipGraph_t gr = nullptr;
    DD_HIP(ctx, hipStreamEndCapture(w->cap, &gr));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return dd_hip_check(ctx, e, "hipGraphInstantiate (coarse GMRES chunk)");
    it = w->graphs.emplace(key, Workspace::Captured{ex, b1 - b0, f1 - f0}).first;
  }
  DD_HIP(ctx, hipGraphLaunch(it->second.exec, st));
  ktimer_account(it->second.bytes, it->second.flops);
  return DD_OK;
}

// Host copies of per-RHS scalars: on the stack up to kHostRhs right-hand sides
// (the allocation-free path stays within that), on the heap beyond.
constexpr int kHostRhs = 64;
template <typename T>
struct HostArr {
  T stack[kHostRhs];
  std::vector<T> heap;
  T* p;
  explicit HostArr(int n, T v = T()) {
    if (n > kHostRhs) {
      heap.assign(n, v);
      p = heap.data();
    } else {
      for (int i = 0; i < n; ++i) stack[i] = v;
      p = stack;
    }
  }
  T& operator[](int i) { return p[i]; }
};

// iteration controls of one even-odd GMRES solve
struct CoarseIter {
  int fixed_iters, max_iters, passes;
  double tol;
};

static CoarseIter coarse_iter(const dd_mg* mg) {
  return {mg->p.coarse_fixed_iters, mg->p.coarse_max_iters, mg->p.coarse_cgs_passes, mg->p.coarse_tol};
}

// y ~= A^-1 b by GMRES on the even-site Schur complement, then the odd sites,
// for the stencil operator A that c describes, on workspace w (coarse part),
// chunks replayed from graphs when `graphs`.
static dd_status coarse_solve_ops(dd_ctx* ctx, Workspace* w, bool graphs, const CoarseOps& c, const CoarseIter& ci,
                                  int nrhs, const void* b, void* y, int* iters_out, hipStream_t st) {
  const dd_dtype vt = c.vt;
  const GeomDev& g = *c.g;
  const int nc = c.nc;
  const long long ld = (long long)g.Vc * nc, ce = (long long)g.Vch * nc;
  const size_t vb = vector_pair_bytes(vt);
  Arnoldi& a = w->ca;
  const int m = a.m;
  const bool fixed = ci.fixed_iters > 0;
  const int cap = fixed ? ci.fixed_iters : ci.max_iters;
  const double tol = fixed ? 0.0 : ci.tol;
  // rhs' = b_e - D_eo D_oo^-1 b_o
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 1, nrhs, g.Vch, g.Vch, 1.0, b, 0.0, nullptr, 0.0, nullptr, w->ct1, st, c.spw, c.bt, c.hm);
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, 0, g.Vch, 0.0, nullptr, -1.0, w->ct1, 1.0, b, w->cr, st, c.spw, c.bt, c.hm);
  DD_HIP(ctx, hipMemsetAsync(y, 0, (size_t)nrhs * ld * vb, st));
  // tolerance: tol * |rhs'|
  norms2(w, vt, nrhs, ce, ld, w->cr, a.nrm2, st);
  {
    HostArr<double2> n2(nrhs);
    HostArr<double> tl(nrhs);
    HostArr<int> fin(nrhs, 0);
    DD_HIP(ctx, hipMemcpyAsync(n2.p, a.nrm2, sizeof(double2) * nrhs, hipMemcpyDeviceToHost, st));
    DD_HIP(ctx, hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) tl[r] = tol * std::sqrt(n2[r].x);
    DD_HIP(ctx, hipMemcpyAsync(a.tolabs, tl.p, sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    DD_HIP(ctx, hipMemcpyAsync(a.finished, fin.p, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    DD_HIP(ctx, hipStreamSynchronize(st));
  }
  const long long vs = (long long)nrhs * ld;   // basis stride
  char* CV = (char*)w->CV;
  if (w->cv_type != c.basis) {
    DD_HIP(ctx, hipMemsetAsync(CV, 0, w->cv_bytes, st));
    w->cv_type = c.basis;
  }
  int iters = 0;
  while (iters < cap) {
    // r = rhs' - S y  (first cycle: y = 0)
    if (iters == 0) {
      DD_HIP(ctx, hipMemcpyAsync(w->cres, w->cr, (size_t)nrhs * ld * vb, hipMemcpyDeviceToDevice, st));
    } else {
      schur_apply(c, nrhs, y, w->cw, w->ct1, w->ct2, st);
      launch_sub(vt, (long long)nrhs * ld, w->cr, w->cw, w->cres, st);
    }
    norms2(w, vt, nrhs, ce, ld, w->cres, a.nrm2, st);
    launch_cycle_init(nrhs, m, a.nrm2, a.tolabs, a.finished, a.gv, a.beta, a.active, a.kcyc, st);
    if (count_active(w, a.active, nrhs, st) == 0) break;
    launch_normalize(vt, nrhs, ce, ld, w->cres, nullptr, a.beta, a.active, CV, st, c.basis,
                     c.basis == DD_F16 ? w->cv32 : nullptr);
    const int mm = (cap - iters < m) ? cap - iters : m;
    // chunks of 4 Arnoldi steps; converged RHS are masked on the device and the
    // host looks between chunks
    for (int j = 0; j < mm;) {
      const int len = mm - j < 4 ? mm - j : 4;
      const bool ends = j + len == mm;
      dd_status cs = run_chunk(ctx, ci.passes, w, graphs, c, nrhs, ce, ld, vs, j, len, ends, st);
      if (cs) return cs;
      iters += len;
      j += len;
      if (ends || count_active(w, a.active, nrhs, st) == 0) break;
    }
    launch_lsq(nrhs, m, a.H, a.gv, a.kcyc, a.y, st);
    launch_multi_axpy(c.basis, vt, nrhs, ce, ld, CV, max_kcyc(w, a, nrhs, st), vs, a.y, m, 0, 1.0, y, st);
    // RHS whose estimate met the tolerance are finished
    DD_HIP(ctx, hipMemcpyAsync(w->hvals, a.est, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    DD_HIP(ctx, hipMemcpyAsync(w->hvals + nrhs, a.tolabs, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    DD_HIP(ctx, hipMemcpyAsync(w->hflags, a.finished, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    DD_HIP(ctx, hipStreamSynchronize(st));
    int nfin = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (w->hvals[r] <= w->hvals[nrhs + r]) w->hflags[r] = 1;
      nfin += w->hflags[r];
    }
    DD_HIP(ctx, hipMemcpyAsync(a.finished, w->hflags, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    if (nfin == nrhs) break;
  }
  // odd sites: y_o = D_oo^-1 (b_o - D_oe y_e)
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, g.Vch, g.Vch, 0.0, nullptr, -1.0, y, 1.0, b, w->ct1, st, c.spw, c.bt, c.hm);
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 1, nrhs, g.Vch, g.Vch, 1.0, w->ct1, 0.0, nullptr, 0.0, nullptr, y, st, c.spw, c.bt, c.hm);
  DD_HIP(ctx, hipGetLastError());
  if (iters_out) *iters_out = iters;
  return DD_OK;
}

// the coarse level's own solve: even-odd GMRES on D_c
static dd_status coarse_solve(dd_mg* mg, Workspace* w, bool graphs, dd_dtype vt, int nrhs, const void* b, void* y,
                              int* iters_out, hipStream_t st) {
  return coarse_solve_ops(mg->ctx, w, graphs, coarse_ops(mg, vt), coarse_iter(mg), nrhs, b, y, iters_out, st);
}

// ---------------------------------------------------------------------------
// third level (kernels in level3.hip): P2, D3 = P2^dag D_c P2, and the coarse
// correction as one flexible GMRES cycle on D_c right preconditioned by
//   M2 v = MR_k(D_c; v, x0 = P2 D3^-1 R2 v),
// D3^-1 being the even-odd GMRES above run on the level-3 lattice.
// ---------------------------------------------------------------------------
struct Level3 {
  dd_level3_params p{};
  int n2 = 0, nc3 = 0, Vc3 = 0;
  int NB3[4] = {0, 0, 0, 0};
  GeomDev g3{};                  // the level-3 lattice as the stencil kernels read it: Vc, Vch, blk_nbr
  std::vector<int> h_lex3;       // lexicographic index of level-3 slot X
  // one allocation: tables, test vectors, P2 and the level-3 blocks
  char* base = nullptr;
  size_t bytes = 0;
  int *nbr3, *slot_of, *l3_of, *loc_of, *flag;
  double2* tv2;                  // [n2][Vc][2n], coarse slot order
  double2* P2_64;                // [Vc3][2][n2][16 n]
  float2* P2_32;
  double2 *D3_64, *Dinv3_64;     // [Vc3][9][col][row], odd sites [Vc3 / 2][col][row]
  float2 *D3_32, *Dinv3_32;      // FP32 copies in the matrix-core order
  dd_dtype half = DD_F64;        // FP16 / BF16 copies as well, for setups that store operands in that type
  void *D3h = nullptr, *Dinv3h = nullptr;
  Workspace* w3 = nullptr;       // level-3 even-odd GMRES
  Workspace* wk = nullptr;       // level-2 FGMRES cycle and its smoother
  int last_steps = 0, last_l3 = 0;
};

static void l3_carve(Level3* L, Arena& a, long long Vc, int n) {
  const long long Vc3 = L->Vc3, nc3 = L->nc3, nvec = (long long)L->n2 * Vc * 2 * n;
  L->nbr3 = a.take<int>(8 * Vc3);
  L->slot_of = a.take<int>(Vc);
  L->l3_of = a.take<int>(Vc);
  L->loc_of = a.take<int>(Vc);
  L->flag = a.take<int>(1);
  L->tv2 = a.take<double2>(nvec);
  L->P2_64 = a.take<double2>(nvec);
  L->P2_32 = a.take<float2>(nvec);
  L->D3_64 = a.take<double2>(Vc3 * 9 * nc3 * nc3);
  L->Dinv3_64 = a.take<double2>(Vc3 / 2 * nc3 * nc3);
  L->D3_32 = a.take<float2>(Vc3 * 9 * nc3 * nc3);
  L->Dinv3_32 = a.take<float2>(Vc3 / 2 * nc3 * nc3);
  if (L->half != DD_F64) {
    L->D3h = a.take<uint32_t>(Vc3 * 9 * nc3 * nc3);
    L->Dinv3h = a.take<uint32_t>(Vc3 / 2 * nc3 * nc3);
  }
}

static void l3_free_ws(dd_mg* mg) {
  Level3* L = mg->l3;
  if (!L) return;
  destroy_ws(mg->ctx, L->w3);
  destroy_ws(mg->ctx, L->wk);
  L->w3 = L->wk = nullptr;
}

static void l3_free(dd_mg* mg) {
  Level3* L = mg->l3;
  if (!L) return;
  l3_free_ws(mg);
  dd_free(mg->ctx, L->base, L->bytes);
  delete L;
  mg->l3 = nullptr;
}

// level-2 FGMRES workspace: D_c z, the smoother's r and D_c r, R2 v and its
// level-3 solve, the Arnoldi basis v_0 .. v_m and the directions z_0 .. z_{m-1}
static void carve_k2(Workspace& w, long long ldc, long long ld3, int nrhs, int m, dd_dtype vt) {
  Arena& a = w.arena;
  const size_t vb = vector_pair_bytes(vt);
  const long long coarse = ldc * nrhs;
  w.cw = a.take<char>(coarse * vb);
  w.cr = a.take<char>(coarse * vb);
  w.ct1 = a.take<char>(coarse * vb);
  w.cb = a.take<char>(ld3 * nrhs * vb);
  w.cy = a.take<char>(ld3 * nrhs * vb);
  w.cv_bytes = (size_t)(m + 1) * coarse * vb;
  w.CV = a.take<char>(w.cv_bytes);
  w.Z = a.take<char>((size_t)m * coarse * vb);
  w.fa.carve(a, nrhs, m);
  w.mr = a.take<double2>(3 * (size_t)nrhs);
  size_t np = (size_t)nrhs * 16 * dots_blocks(ldc, nrhs) * 2;
  const size_t np_gs = (size_t)nrhs * m * gs_blocks(ldc) * 2;
  w.partial = a.take<double>(std::max(np, np_gs));
}

static dd_status l3_ensure_ws(dd_mg* mg, int nrhs) {
  Level3* L = mg->l3;
  if (L->w3 && L->w3->nrhs >= nrhs) return DD_OK;
  if (L->w3 && L->w3->nrhs > nrhs) nrhs = L->w3->nrhs;
  l3_free_ws(mg);
  const dd_dtype vt = inner_vt(mg);
  const WsShape s3{0, L->Vc3, L->Vc3 / 2, L->nc3, L->p.l3_restart, 1, vt};
  dd_status s = alloc_ws(mg->ctx, nrhs, [&](Workspace& x) { carve_ws(x, s3, nrhs, false, false); }, &L->w3);
  if (s) return s;
  const long long ldc = (long long)mg->g->geo.Vc * mg->nc, ld3 = (long long)L->Vc3 * L->nc3;
  s = alloc_ws(mg->ctx, nrhs, [&](Workspace& x) { carve_k2(x, ldc, ld3, nrhs, L->p.kcycle_max_iters, vt); }, &L->wk);
  if (s) l3_free_ws(mg);
  return s;
}

// the level-3 stencil as the even-odd GMRES applies it; the coarse arithmetic
// choices of the gauge field's tuning hold for it as for D_c
static CoarseOps l3_ops(const dd_mg* mg, dd_dtype vt) {
  const Level3* L = mg->l3;
  const Tuning& t = mg->g->tune;
  const bool half = vt == DD_F32 && L->D3h && t.coarse_half;
  CoarseOps c;
  c.g = &L->g3;
  c.vt = vt;
  c.nc = L->nc3;
  c.Dc = vt == DD_F64 ? (const void*)L->D3_64 : half ? L->D3h : (const void*)L->D3_32;
  c.Dinv = vt == DD_F64 ? (const void*)L->Dinv3_64 : half ? L->Dinv3h : (const void*)L->Dinv3_32;
  c.spw = t.coarse_spw;
  c.bt = vt == DD_F64 ? DD_F64 : half ? L->half : DD_F32;
  c.hm = half && t.coarse_mfma_half;
  c.basis = (vt == DD_F32 && t.coarse_basis_half) ? DD_F16 : vt;
  c.bb = c.basis == DD_F16 ? sizeof(__half2) : vector_pair_bytes(vt);
  return c;
}

// z = M2 v on the level-2 workspace; *it3 <- level-3 GMRES steps.  With MR
// steps, w->cr ends as the smoother's residual v - D_c z (updated recursively).
static dd_status precond2(dd_mg* mg, dd_dtype vt, int nrhs, const void* v, void* z, int* it3, hipStream_t st) {
  Level3* L = mg->l3;
  Workspace* w = L->wk;
  const GeomDev& g = mg->g->geo;
  const int nc = mg->nc, n = mg->n;
  const long long ld = (long long)g.Vc * nc;
  const void* P2 = vt == DD_F64 ? (const void*)L->P2_64 : (const void*)L->P2_32;
  launch_restrict2(vt, g.Vc, L->Vc3, n, L->n2, L->slot_of, P2, nrhs, v, w->cb, st);
  const CoarseIter ci{L->p.l3_fixed_iters, L->p.l3_max_iters, mg->p.coarse_cgs_passes, L->p.l3_tol};
  dd_status s = coarse_solve_ops(mg->ctx, L->w3, mg->graphs >= 1, l3_ops(mg, vt), ci, nrhs, w->cb, w->cy, it3, st);
  if (s) return s;
  launch_prolong2(vt, g.Vc, L->Vc3, n, L->n2, L->l3_of, L->loc_of, P2, nrhs, w->cy, z, st);
  if (L->p.mr_steps == 0) return DD_OK;
  const CoarseOps c = coarse_ops(mg, vt);
  // r = v - D_c z, then per step: alpha = <D_c r, r> / <D_c r, D_c r>, z += alpha r, r -= alpha D_c r
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, 0, g.Vc, -1.0, z, -1.0, z, 1.0, v, w->cr, st, c.spw, c.bt, c.hm);
  double2 *num = w->mr, *den = w->mr + nrhs, *alpha = w->mr + 2 * nrhs;
  const int nblk = dots_blocks(ld, nrhs);
  for (int k = 0; k < L->p.mr_steps; ++k) {
    launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, 0, g.Vc, 1.0, w->cr, 1.0, w->cr, 0.0, nullptr, w->ct1, st,
                     c.spw, c.bt, c.hm);
    launch_dots(vt, vt, nrhs, ld, ld, w->ct1, 1, 0, w->cr, w->partial, nblk, num, 1, 0, st);
    launch_dots(vt, vt, nrhs, ld, ld, w->ct1, 1, 0, w->ct1, w->partial, nblk, den, 1, 0, st);
    launch_mr_alpha(nrhs, num, den, alpha, st);
    launch_multi_axpy(vt, vt, nrhs, ld, ld, w->cr, 1, 0, alpha, 1, 0, 1.0, z, st);
    launch_multi_axpy(vt, vt, nrhs, ld, ld, w->ct1, 1, 0, alpha, 1, 0, -1.0, w->cr, st);
  }
  return DD_OK;
}

// y ~= D_c^-1 b: one flexible GMRES cycle from y = 0, right preconditioned by M2
static dd_status kcycle_solve(dd_mg* mg, dd_dtype vt, int nrhs, const void* b, void* y, int* iters_out,
                              hipStream_t st) {
  Level3* L = mg->l3;
  dd_status s = l3_ensure_ws(mg, nrhs);
  if (s) return s;
  Workspace* w = L->wk;
  const GeomDev& g = mg->g->geo;
  const int nc = mg->nc;
  const long long ld = (long long)g.Vc * nc, vs = (long long)nrhs * ld;
  const size_t vb = vector_pair_bytes(vt);
  const CoarseOps c = coarse_ops(mg, vt);
  Arnoldi& a = w->fa;
  const int m = a.m;
  const double tol = L->p.kcycle_fixed ? 0.0 : L->p.kcycle_tol;
  char *V = (char*)w->CV, *Z = (char*)w->Z;
  norms2(w, vt, nrhs, ld, ld, b, a.nrm2, st);
  {
    HostArr<double2> n2(nrhs);
    HostArr<double> tl(nrhs);
    HostArr<int> fin(nrhs, 0);
    DD_HIP(mg->ctx, hipMemcpyAsync(n2.p, a.nrm2, sizeof(double2) * nrhs, hipMemcpyDeviceToHost, st));
    DD_HIP(mg->ctx, hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) tl[r] = tol * std::sqrt(n2[r].x);
    DD_HIP(mg->ctx, hipMemcpyAsync(a.tolabs, tl.p, sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    DD_HIP(mg->ctx, hipMemcpyAsync(a.finished, fin.p, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    DD_HIP(mg->ctx, hipStreamSynchronize(st));
  }
  launch_cycle_init(nrhs, m, a.nrm2, a.tolabs, a.finished, a.gv, a.beta, a.active, a.kcyc, st);
  launch_zero(y, (size_t)nrhs * ld * vb, st);
  int steps = 0, total3 = 0;
  if (count_active(w, a.active, nrhs, st) > 0) {
    launch_normalize(vt, nrhs, ld, ld, b, nullptr, a.beta, a.active, V, st, vt);
    for (int j = 0; j < m; ++j) {
      char* Vj = V + (size_t)j * vs * vb;
      char* Zj = Z + (size_t)j * vs * vb;
      int it3 = 0;
      if ((s = precond2(mg, vt, nrhs, Vj, Zj, &it3, st))) return s;
      total3 += it3;
      // w = D_c z_j: after MR steps it is v_j - r, the smoother's residual carried along (one stencil
      // apply fewer per step; the recursion's rounding is far below the cycle's tolerance)
      if (L->p.mr_steps > 0)
        launch_sub(vt, vs, Vj, w->cr, w->cw, st);
      else
        launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, 0, g.Vc, 1.0, Zj, 1.0, Zj, 0.0, nullptr, w->cw, st, c.spw,
                         c.bt, c.hm);
      cgs(w, a, vt, nrhs, ld, ld, V, vs, j + 1, w->cw, 1, st, vt);
      launch_arnoldi(nrhs, m, j, a.h1, nullptr, a.nrm2, a.H, a.cs, a.sn, a.gv, a.tolabs, a.active, a.kcyc, a.est,
                     a.hnext, st);
      steps = j + 1;
      if (j + 1 == m) break;
      launch_normalize(vt, nrhs, ld, ld, w->cw, nullptr, a.hnext, a.active, V + (size_t)(j + 1) * vs * vb, st, vt);
      if (count_active(w, a.active, nrhs, st) == 0) break;
    }
    launch_lsq(nrhs, m, a.H, a.gv, a.kcyc, a.y, st);
    launch_multi_axpy(vt, vt, nrhs, ld, ld, Z, max_kcyc(w, a, nrhs, st), vs, a.y, m, 0, 1.0, y, st);
  }
  DD_HIP(mg->ctx, hipGetLastError());
  L->last_steps = steps;
  L->last_l3 = total3;
  if (iters_out) *iters_out = steps;
  return DD_OK;
}

// the coarse correction's solve: two-level GMRES, or the level-2 cycle when a third level is attached
static dd_status coarse_correction(dd_mg* mg, Workspace* w, bool graphs, dd_dtype vt, int nrhs, const void* b,
                                   void* y, int* iters_out, hipStream_t st) {
  if (mg->l3) return kcycle_solve(mg, vt, nrhs, b, y, iters_out, st);
  return coarse_solve(mg, w, graphs, vt, nrhs, b, y, iters_out, st);
}

// P2 from the level-2 test vectors, then D3 and its odd-site inverses
static dd_status l3_build(dd_mg* mg, hipStream_t st) {
  Level3* L = mg->l3;
  const GeomDev& G = mg->g->geo;
  const int neg = -1;
  int bad = -1;
  DD_HIP(mg->ctx, hipMemcpyAsync(L->flag, &neg, sizeof(int), hipMemcpyHostToDevice, st));
  launch_gs2(G.Vc, L->Vc3, mg->n, L->n2, L->slot_of, L->tv2, L->P2_64, L->flag, st);
  DD_HIP(mg->ctx, hipMemcpyAsync(&bad, L->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  if (bad >= 0)
    return dd_fail(mg->ctx, DD_EINVAL,
                   "level-2 test vectors are rank deficient on level-3 site " + std::to_string(L->h_lex3[bad / 2]) +
                       " chirality " + std::to_string(bad % 2));
  const long long nvec = (long long)L->n2 * G.Vc * mg->nc;
  launch_convert_pairs(DD_F32, L->P2_64, nullptr, L->P2_32, nvec, st);
  return DD_OK;
}

static dd_status l3_galerkin(dd_mg* mg, hipStream_t st) {
  Level3* L = mg->l3;
  const GeomDev& G = mg->g->geo;
  const int neg = -1, nc3 = L->nc3;
  int bad = -1;
  launch_galerkin3(G, L->Vc3, mg->n, L->n2, L->slot_of, L->l3_of, L->loc_of, mg->Dc64, L->P2_64, L->D3_64, st);
  DD_HIP(mg->ctx, hipMemcpyAsync(L->flag, &neg, sizeof(int), hipMemcpyHostToDevice, st));
  launch_coarse_invert(L->g3, nc3, L->D3_64, L->Dinv3_64, L->flag, st);
  launch_coarse_tile(nc3, L->D3_64, 9LL * L->Vc3, L->D3_32, L->half, L->D3h, st);
  launch_coarse_tile(nc3, L->Dinv3_64, L->Vc3 / 2, L->Dinv3_32, L->half, L->Dinv3h, st);
  DD_HIP(mg->ctx, hipMemcpyAsync(&bad, L->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  DD_HIP(mg->ctx, hipGetLastError());
  if (bad >= 0)
    return dd_fail(mg->ctx, DD_EINVAL, "singular level-3 self block on level-3 site " + std::to_string(L->h_lex3[bad]));
  return DD_OK;
}

// ---------------------------------------------------------------------------
// preconditioner M (Eq. 5): x_c = P D_c^-1 R v, then SAP on D x = v from x_c
// ---------------------------------------------------------------------------
static dd_status vcycle(dd_mg* mg, int nrhs, const void* v, void* out, int* citers, hipStream_t st) {
  Workspace* w = mg->ws;
  dd_dtype vt = inner_vt(mg);
  const GeomDev& g = mg->g->geo;
  launch_restrict(g, vt, P_inner_dt(mg), mg->n, P_inner(mg), nrhs, v, w->cb, st);
  dd_status s = coarse_correction(mg, w, mg->graphs == 1, vt, nrhs, w->cb, w->cy, citers, st);
  if (s) return s;
  launch_prolong(g, vt, P_inner_dt(mg), mg->n, P_inner(mg), nrhs, w->cy, out, st);
  dd_dtype od = op_dtype(mg);
  launch_sap(g, od, mg->g->ops[od], nrhs, mg->p.sap_sweeps, mg->p.sap_mr_iters, v, out, mg->g->tune.sap_wpe,
             mg->g->tune.sap_dom_rhs, mg->g->tune.sap_persist, st);
  DD_HIP(mg->ctx, hipGetLastError());
  return DD_OK;
}

// ---------------------------------------------------------------------------
// M without host round trips (graph mode 2): the coarse GMRES decides on the
// device when each right-hand side is done.  The launches are those of
// coarse_solve, in the same order, for a fixed number of steps (the iteration
// cap, in cycles of the restart length from steps 0, m, 2m, ...); gates make a
// step's kernels return at once when no right-hand side is active in it, and a
// cycle's residual and update kernels when every right-hand side is finished.
// A masked right-hand side is never written, the basis update runs over the
// whole cycle with zero coefficients past a right-hand side's own steps, so the
// result equals the host-checked solve bit for bit (the cycle boundaries differ
// only after an exact breakdown of the Arnoldi process, h = 0, which the host
// form would follow by a shorter cycle).
// ---------------------------------------------------------------------------
static void coarse_solve_device(dd_mg* mg, Workspace* w, dd_dtype vt, int nrhs, const void* b, void* y,
                                hipStream_t st) {
  CoarseOps c = coarse_ops(mg, vt);
  const GeomDev& g = *c.g;
  const int nc = c.nc;
  const long long ld = (long long)g.Vc * nc, ce = (long long)g.Vch * nc;
  const size_t vb = vector_pair_bytes(vt);
  Arnoldi& a = w->ca;
  const int m = a.m;
  const bool fixed = mg->p.coarse_fixed_iters > 0;
  const int cap = fixed ? mg->p.coarse_fixed_iters : mg->p.coarse_max_iters;
  const double tol = fixed ? 0.0 : mg->p.coarse_tol;
  const int passes = mg->p.coarse_cgs_passes;
  const long long vs = (long long)nrhs * ld;
  char* CV = (char*)w->CV;
  // rhs' = b_e - D_eo D_oo^-1 b_o; y = 0; tolerance from |rhs'| (all on the device)
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 1, nrhs, g.Vch, g.Vch, 1.0, b, 0.0, nullptr, 0.0, nullptr, w->ct1, st, c.spw, c.bt, c.hm);
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, 0, g.Vch, 0.0, nullptr, -1.0, w->ct1, 1.0, b, w->cr, st, c.spw, c.bt, c.hm);
  launch_zero(y, (size_t)nrhs * ld * vb, st);
  norms2(w, vt, nrhs, ce, ld, w->cr, a.nrm2, st);
  launch_set_tol(nrhs, tol, a.nrm2, a.tolabs, a.finished, a.active, st);
  const Gate unfinished{a.finished, nrhs, 0}, active{a.active, nrhs, 1};
  for (int c0 = 0; c0 < cap; c0 += m) {
    const int mm = cap - c0 < m ? cap - c0 : m;
    {
      GateScope gs(unfinished);
      if (c0 == 0) {
        launch_copy(vt, (long long)nrhs * ld, w->cr, w->cres, st);
      } else {
        schur_apply(c, nrhs, y, w->cw, w->ct1, w->ct2, st);
        launch_sub(vt, (long long)nrhs * ld, w->cr, w->cw, w->cres, st);
      }
      norms2(w, vt, nrhs, ce, ld, w->cres, a.nrm2, st);
      launch_cycle_init(nrhs, m, a.nrm2, a.tolabs, a.finished, a.gv, a.beta, a.active, a.kcyc, st);
    }
    {
      GateScope ga(active);
      launch_normalize(vt, nrhs, ce, ld, w->cres, nullptr, a.beta, a.active, CV, st, c.basis,
                       c.basis == DD_F16 ? w->cv32 : nullptr);
      issue_chunk(c, w, a, passes, nrhs, ce, ld, vs, CV, 0, mm, true, st);
    }
    {
      GateScope gs(unfinished);
      launch_lsq(nrhs, m, a.H, a.gv, a.kcyc, a.y, st);
      launch_multi_axpy(c.basis, vt, nrhs, ce, ld, CV, mm, vs, a.y, m, 0, 1.0, y, st);
      launch_finish(nrhs, a.est, a.tolabs, a.finished, a.active, a.kcyc, w->citers, st);
    }
  }
  // odd sites: y_o = D_oo^-1 (b_o - D_oe y_e)
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 0, nrhs, g.Vch, g.Vch, 0.0, nullptr, -1.0, y, 1.0, b, w->ct1, st, c.spw, c.bt, c.hm);
  launch_coarse_mv(g, vt, nc, c.Dc, c.Dinv, 1, nrhs, g.Vch, g.Vch, 1.0, w->ct1, 0.0, nullptr, 0.0, nullptr, y, st, c.spw, c.bt, c.hm);
}

// M v as one graph: restriction, the device-driven coarse solve, prolongation
// and SAP, captured on first use per (nrhs, choices, buffers) and replayed.
static dd_status vcycle_graph(dd_mg* mg, int nrhs, const void* v, void* out, hipStream_t st) {
  Workspace* w = mg->ws;
  const dd_dtype vt = inner_vt(mg);
  const CoarseOps c = coarse_ops(mg, vt);
  const Tuning& t = mg->g->tune;
  const std::array<long long, 12> key = {nrhs, (long long)vt, (long long)c.basis, (long long)c.bt, c.spw, c.hm ? 1 : 0,
                                         t.sap_wpe, t.sap_dom_rhs, (long long)(intptr_t)v, (long long)(intptr_t)out,
                                         mg->p.coarse_max_iters, mg->p.coarse_fixed_iters};
  auto it = w->mgraphs.find(key);
  if (it == w->mgraphs.end()) {
    if (w->cv_type != c.basis) {   // clear the basis outside the capture (no fill nodes recorded)
      launch_zero(w->CV, w->cv_bytes, st);
      w->cv_type = c.basis;
    }
    if (w->mgraphs.size() >= 64) {   // callers cycling through many buffers: start over
      for (auto& kv : w->mgraphs) (void)hipGraphExecDestroy(kv.second.exec);
      w->mgraphs.clear();
    }
    if (!w->cap) DD_HIP(mg->ctx, hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking));
    DD_HIP(mg->ctx, hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
    double b0, f0, b1, f1;
    ktimer_model(&b0, &f0);
    ktimer_suspend(true);
    const GeomDev& g = mg->g->geo;
    launch_restrict(g, vt, P_inner_dt(mg), mg->n, P_inner(mg), nrhs, v, w->cb, w->cap);
    coarse_solve_device(mg, w, vt, nrhs, w->cb, w->cy, w->cap);
    launch_prolong(g, vt, P_inner_dt(mg), mg->n, P_inner(mg), nrhs, w->cy, out, w->cap);
    const dd_dtype od = op_dtype(mg);
    launch_sap(g, od, mg->g->ops[od], nrhs, mg->p.sap_sweeps, mg->p.sap_mr_iters, v, out, t.sap_wpe, t.sap_dom_rhs,
               0, w->cap);   // captured: the launch form
    ktimer_suspend(false);
    ktimer_model(&b1, &f1);
    ktimer_model_set(b0, f0);
    hipGraph_t gr = nullptr;
    DD_HIP(mg->ctx, hipStreamEndCapture(w->cap, &gr));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return dd_hip_check(mg->ctx, e, "hipGraphInstantiate (preconditioner)");
    it = w->mgraphs.emplace(key, Workspace::Captured{ex, b1 - b0, f1 - f0}).first;
  }
  DD_HIP(mg->ctx, hipGraphLaunch(it->second.exec, st));
  ktimer_account(it->second.bytes, it->second.flops);
  return DD_OK;
}

// M as one graph (mode 2; with a third level, whose GMRES checks convergence on the host, mode 2 runs as mode 1)
static bool whole_graph(const dd_mg* mg) { return mg->graphs == 2 && !mg->l3; }

// M v in the mode the setup is in
static dd_status apply_M(dd_mg* mg, int nrhs, const void* v, void* out, int* citers, hipStream_t st) {
  if (whole_graph(mg)) {
    if (citers) *citers = 0;   // counted on the device (Workspace::citers)
    return vcycle_graph(mg, nrhs, v, out, st);
  }
  return vcycle(mg, nrhs, v, out, citers, st);
}

// ---------------------------------------------------------------------------
// build: Gram-Schmidt, stored P, D_c = P^dag D P, odd-site inverses
// ---------------------------------------------------------------------------
static dd_status build(dd_mg* mg, hipStream_t st) {
  dd_gauge* g = mg->g;
  const GeomDev& G = g->geo;
  const long long nfine = 12LL * G.V * mg->n;
  int* dflag = nullptr;
  dd_status s;
  if ((s = dd_alloc(mg->ctx, (void**)&dflag, sizeof(int)))) return s;
  int neg = -1;
  // P64 <- working vectors
  launch_vec_convert(inner_vt(mg), DD_F64, mg->tv, mg->P64, nfine, st);
  DD_HIP(mg->ctx, hipMemcpyAsync(dflag, &neg, sizeof(int), hipMemcpyHostToDevice, st));
  launch_gram_schmidt(G, mg->n, mg->P64, dflag, st);
  int bad = -1;
  DD_HIP(mg->ctx, hipMemcpyAsync(&bad, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  if (bad >= 0) {
    dd_free(mg->ctx, dflag, sizeof(int));
    return dd_fail(mg->ctx, DD_EINVAL,
                   "test vectors are rank deficient on aggregate slot " + std::to_string(bad / 2) + " chirality " +
                       std::to_string(bad % 2));
  }
  // stored copy of P: FP32 from FP64, half precision from the FP32 copy
  if (mg->vstore != DD_F64) {
    if (mg->vstore == DD_F32) {
      launch_convert_pairs(DD_F32, mg->P64, nullptr, mg->Pst, nfine, st);
    } else {
      // through an FP32 staging buffer of at most 2^27 pairs (1 GiB), chunk by chunk
      const long long cap = 1LL << 27, len = nfine < cap ? nfine : cap;
      float2* stage = nullptr;
      if ((s = dd_alloc(mg->ctx, (void**)&stage, sizeof(float2) * len))) {
        dd_free(mg->ctx, dflag, sizeof(int));
        return s;
      }
      const size_t pb = storage_pair_bytes(mg->vstore);
      for (long long o = 0; o < nfine; o += len) {
        const long long cnt = nfine - o < len ? nfine - o : len;
        launch_convert_pairs(DD_F32, mg->P64 + o, nullptr, stage, cnt, st);
        launch_convert_pairs(mg->vstore, nullptr, stage, (char*)mg->Pst + o * pb, cnt, st);
      }
      DD_HIP(mg->ctx, hipStreamSynchronize(st));
      dd_free(mg->ctx, stage, sizeof(float2) * len);
    }
  }
  // Galerkin operator from the stored P and the FP64 operator.  W holds `chunk`
  // FP64 fine vectors (columns of D_c built per pass over P): as many as fit in
  // 4 GiB, or in half of the budget still free up to 32 GiB, whichever is larger,
  // rounded down to whole 16-column passes of the restriction.  Every column is
  // computed on its own, so the chunk changes the number of passes, not the result.
  const long long vbytes = 12LL * G.V * (long long)sizeof(double2);
  const size_t used = ctx_in_use(mg->ctx), free_b = mg->ctx->budget > used ? mg->ctx->budget - used : 0;
  const size_t wcap = std::max<size_t>(4ULL << 30, std::min<size_t>(free_b / 2, 32ULL << 30));
  int chunk = (int)std::min<long long>((long long)(wcap / (size_t)vbytes), mg->nc);
  if (chunk >= 16 && chunk < mg->nc) chunk -= chunk % 16;
  if (chunk < 1) chunk = 1;
  double2* W = nullptr;
  if ((s = dd_alloc(mg->ctx, (void**)&W, (size_t)chunk * vbytes))) {
    dd_free(mg->ctx, dflag, sizeof(int));
    return s;
  }
  const void* Pb = mg->vstore == DD_F64 ? (const void*)mg->P64 : mg->Pst;
  launch_coarse_build(G, g->ops[DD_F64], mg->vstore, mg->n, Pb, mg->Dc64, W, chunk, st);
  DD_HIP(mg->ctx, hipMemcpyAsync(dflag, &neg, sizeof(int), hipMemcpyHostToDevice, st));
  launch_coarse_invert(G, mg->nc, mg->Dc64, mg->Dinv64, dflag, st);
  const long long ndc = (long long)G.Vc * 9 * mg->nc * mg->nc, ndi = (long long)G.Vch * mg->nc * mg->nc;
  // FP32 copies (and half copies rounded from them) in the matrix-core order
  const dd_dtype half = mg->Dch ? mg->vstore : DD_F64;
  const long long nn = (long long)mg->nc * mg->nc;
  launch_coarse_tile(mg->nc, mg->Dc64, ndc / nn, mg->Dc32, half, mg->Dch, st);
  launch_coarse_tile(mg->nc, mg->Dinv64, ndi / nn, mg->Dinv32, half, mg->Dinvh, st);
  DD_HIP(mg->ctx, hipMemcpyAsync(&bad, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  dd_free(mg->ctx, W, (size_t)chunk * vbytes);
  dd_free(mg->ctx, dflag, sizeof(int));
  if (bad >= 0) return dd_fail(mg->ctx, DD_EINVAL, "singular coarse self block on coarse slot " + std::to_string(bad));
  return DD_OK;
}

// lambda_i <- lambda_i / |lambda_i|
static void normalize_vectors(dd_mg* mg, void* tv, hipStream_t st) {
  Workspace* w = mg->ws;
  const long long cnt = 12LL * mg->g->geo.V;
  norms2(w, inner_vt(mg), mg->n, cnt, cnt, tv, w->ca.nrm2, st);
  launch_normalize(inner_vt(mg), mg->n, cnt, cnt, tv, w->ca.nrm2, nullptr, nullptr, tv, st);
}

static size_t mg_bytes_P64(const dd_mg* mg) { return 16ULL * 12 * mg->g->geo.V * mg->n; }
static size_t mg_bytes_tv(const dd_mg* mg) { return vector_pair_bytes(inner_vt(mg)) * 12ULL * mg->g->geo.V * mg->n; }
static size_t mg_bytes_Pst(const dd_mg* mg) {
  return mg->vstore == DD_F64 ? 0 : storage_pair_bytes(mg->vstore) * 12ULL * mg->g->geo.V * mg->n;
}
static size_t mg_bytes_Dc(const dd_mg* mg, size_t pb) { return pb * mg->g->geo.Vc * 9ULL * mg->nc * mg->nc; }
static size_t mg_bytes_Dinv(const dd_mg* mg, size_t pb) { return pb * mg->g->geo.Vch * 1ULL * mg->nc * mg->nc; }

static void mg_free(dd_mg* mg) {
  l3_free(mg);
  free_ws(mg);
  dd_free(mg->ctx, mg->P64, mg_bytes_P64(mg));
  dd_free(mg->ctx, mg->tv, mg_bytes_tv(mg));
  dd_free(mg->ctx, mg->Pst, mg_bytes_Pst(mg));
  dd_free(mg->ctx, mg->Dc64, mg_bytes_Dc(mg, 16));
  dd_free(mg->ctx, mg->Dc32, mg_bytes_Dc(mg, 8));
  dd_free(mg->ctx, mg->Dinv64, mg_bytes_Dinv(mg, 16));
  dd_free(mg->ctx, mg->Dinv32, mg_bytes_Dinv(mg, 8));
  dd_free(mg->ctx, mg->Dch, mg_bytes_Dc(mg, 4));
  dd_free(mg->ctx, mg->Dinvh, mg_bytes_Dinv(mg, 4));
  if (mg->g) mg->g->refcount--;
  delete mg;
}

static dd_status validate_params(dd_gauge* g, const dd_mg_params* p) {
  for (int m = 0; m < 4; ++m)
    if (p->agg_block[m] != g->prob.block[m] || p->sap_block[m] != g->prob.block[m])
      return dd_fail(g->ctx, DD_ESHAPE, "aggregate and SAP blocks must equal the gauge field's block tiling");
  if (p->n_vec % 2) return dd_fail(g->ctx, DD_ESHAPE, "n_vec must be even (Sec. 3)");
  if (!supported_nvec(p->n_vec)) return dd_fail(g->ctx, DD_ESHAPE, "n_vec must be one of 6, 8, 12, 16, 20, 24");
  if (p->sap_sweeps < 0 || p->sap_mr_iters < 0 || p->setup_iters < 0 || p->init_sap_apps < 0)
    return dd_fail(g->ctx, DD_EINVAL, "negative iteration counts");
  if (p->coarse_restart < 1 || p->coarse_restart > 256 || p->fgmres_restart < 1 || p->fgmres_restart > 64)
    return dd_fail(g->ctx, DD_EINVAL, "coarse restart must be in [1, 256], FGMRES restart in [1, 64]");
  if (p->coarse_max_iters < 1 || p->max_outer_iters < 1) return dd_fail(g->ctx, DD_EINVAL, "iteration caps must be >= 1");
  if (p->coarse_cgs_passes != 1 && p->coarse_cgs_passes != 2)
    return dd_fail(g->ctx, DD_EINVAL, "coarse_cgs_passes must be 1 or 2");
  if (p->outer_cgs_passes != 1 && p->outer_cgs_passes != 2)
    return dd_fail(g->ctx, DD_EINVAL, "outer_cgs_passes must be 1 or 2");
  if (p->inner_dtype != DD_F64 && p->inner_dtype != DD_F32)
    return dd_fail(g->ctx, DD_EINVAL, "inner_dtype must be DD_F64 or DD_F32");
  if ((int)p->store_dtype < 0 || (int)p->store_dtype > 3) return dd_fail(g->ctx, DD_EINVAL, "unknown store_dtype");
  if (p->inner_dtype == DD_F32 && p->store_dtype == DD_F64)
    return dd_fail(g->ctx, DD_EINVAL, "FP32 inner solvers take FP32, FP16 or BF16 stored operands");
  if (p->inner_dtype == DD_F64 && p->store_dtype != DD_F64)
    return dd_fail(g->ctx, DD_EINVAL, "the all-FP64 preconditioner needs store_dtype DD_F64");
  return DD_OK;
}

static dd_status setup_common(dd_gauge* g, const dd_mg_params* p, const double* tv_host, dd_mg** out) {
  if (!g || !p || !out) return DD_EINVAL;
  *out = nullptr;
  dd_status s = validate_params(g, p);
  if (s) return s;
  hipStream_t st = 0;
  dd_mg* mg = new dd_mg();
  mg->ctx = g->ctx;
  mg->g = g;
  g->refcount++;
  mg->p = *p;
  mg->n = p->n_vec;
  mg->nc = 2 * p->n_vec;
  mg->vstore = p->inner_dtype == DD_F64 ? DD_F64 : p->store_dtype;
  auto fail = [&](dd_status e) {
    mg_free(mg);
    return e;
  };
  dd_dtype od = op_dtype(mg);
  if ((s = ensure_opset(g, od))) return fail(s);
  if ((s = dd_alloc(mg->ctx, (void**)&mg->P64, mg_bytes_P64(mg))) ||
      (s = dd_alloc(mg->ctx, (void**)&mg->tv, mg_bytes_tv(mg))) ||
      (s = dd_alloc(mg->ctx, (void**)&mg->Pst, mg_bytes_Pst(mg))) ||
      (s = dd_alloc(mg->ctx, (void**)&mg->Dc64, mg_bytes_Dc(mg, 16))) ||
      (s = dd_alloc(mg->ctx, (void**)&mg->Dc32, mg_bytes_Dc(mg, 8))) ||
      (s = dd_alloc(mg->ctx, (void**)&mg->Dinv64, mg_bytes_Dinv(mg, 16))) ||
      (s = dd_alloc(mg->ctx, (void**)&mg->Dinv32, mg_bytes_Dinv(mg, 8))))
    return fail(s);
  if ((mg->vstore == DD_F16 || mg->vstore == DD_BF16) &&
      ((s = dd_alloc(mg->ctx, &mg->Dch, mg_bytes_Dc(mg, 4))) ||
       (s = dd_alloc(mg->ctx, &mg->Dinvh, mg_bytes_Dinv(mg, 4)))))
    return fail(s);
  if ((s = ensure_ws(mg, mg->n, false))) return fail(s);
  const GeomDev& G = g->geo;
  const long long nfine = 12LL * G.V * mg->n;
  // starting vectors, canonical FP64 -> packed working dtype.  P64 (exactly n
  // canonical FP64 fine vectors in size) is the staging buffer: build()
  // overwrites it with the orthonormalised vectors, so the setup allocates no
  // second copy.
  double2* canon = mg->P64;
  if (tv_host) {
    hipError_t e = hipMemcpy(canon, tv_host, sizeof(double2) * nfine, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(dd_hip_check(mg->ctx, e, "test vector upload"));
  } else {
    launch_gauss(p->seed, nfine, canon, st);
  }
  launch_pack_fine(G, inner_vt(mg), mg->n, canon, mg->tv, st);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(dd_hip_check(mg->ctx, e, "starting vectors"));
  Workspace* w = mg->ws;
  const size_t fb = vector_pair_bytes(inner_vt(mg)) * (size_t)nfine;
  // initial approximate solves: lambda_i <- SAP(b = lambda_i, x0 = 0)
  for (int k = 0; k < p->init_sap_apps; ++k) {
    DD_HIP(mg->ctx, hipMemcpyAsync(w->vin, mg->tv, fb, hipMemcpyDeviceToDevice, st));
    DD_HIP(mg->ctx, hipMemsetAsync(mg->tv, 0, fb, st));
    launch_sap(G, od, g->ops[od], mg->n, p->sap_sweeps, p->sap_mr_iters, w->vin, mg->tv, g->tune.sap_wpe,
               g->tune.sap_dom_rhs, g->tune.sap_persist, st);
    normalize_vectors(mg, mg->tv, st);
  }
  if ((s = build(mg, st))) return fail(s);
  // adaptive iterations: lambda_i <- M lambda_i, normalise, rebuild
  for (int k = 0; k < p->setup_iters; ++k) {
    DD_HIP(mg->ctx, hipMemcpyAsync(w->xs, mg->tv, fb, hipMemcpyDeviceToDevice, st));
    if ((s = vcycle(mg, mg->n, w->xs, mg->tv, nullptr, st))) return fail(s);
    normalize_vectors(mg, mg->tv, st);
    if ((s = build(mg, st))) return fail(s);
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(dd_hip_check(mg->ctx, e, "setup"));
  free_ws(mg);   // the solve sizes its own workspace for its number of right-hand sides
  *out = mg;
  return DD_OK;
}

static dd_status check_mg_vec(dd_mg* mg, dd_dtype dt, int nrhs, const void* a, const void* b) {
  if (!mg) return DD_EINVAL;
  if (dt != DD_F64 && dt != DD_F32) return dd_fail(mg->ctx, DD_EINVAL, "coarse-level dtype must be DD_F64 or DD_F32");
  if (!a || !b || nrhs < 1) return dd_fail(mg->ctx, DD_EINVAL, "bad vector arguments");
  if (a == b) return dd_fail(mg->ctx, DD_EINVAL, "input and output must not alias");
  return DD_OK;
}

// ---------------------------------------------------------------------------
// autotuner cache: a JSON object, one entry per line,
//   "<device>|L=..|b=..|n=..|nrhs=..|op=..|inner=..|cblk=..":
//       {"sap_wpe": 2, "sap_dom_rhs": 4, "sap_persist": 0, "dirac_threads": 256, "coarse_spw": 4}
// (launch shapes only; the coarse arithmetic choices are the caller's and part of the key)
// Lines that do not parse are dropped (the file is rewritten on the next miss).
// ---------------------------------------------------------------------------
static bool tune_field(const std::string& obj, const char* name, int& v) {
  std::string pat = std::string("\"") + name + "\":";
  size_t p = obj.find(pat);
  if (p == std::string::npos) return false;
  return std::sscanf(obj.c_str() + p + pat.size(), " %d", &v) == 1;
}

static void tune_cache_read(const char* path, std::map<std::string, Tuning>& out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char buf[1024];
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string l(buf);
    size_t a = l.find('"'), b = a == std::string::npos ? a : l.find('"', a + 1);
    size_t o = b == std::string::npos ? b : l.find('{', b), c = o == std::string::npos ? o : l.find('}', o);
    if (c == std::string::npos) continue;
    std::string obj = l.substr(o, c - o + 1);
    Tuning t;
    if (tune_field(obj, "sap_wpe", t.sap_wpe) && tune_field(obj, "sap_dom_rhs", t.sap_dom_rhs) &&
        tune_field(obj, "sap_persist", t.sap_persist) && tune_field(obj, "dirac_threads", t.dirac_threads) &&
        tune_field(obj, "coarse_spw", t.coarse_spw))
      out[l.substr(a + 1, b - a - 1)] = t;
  }
  std::fclose(f);
}

static bool tune_cache_write(const char* path, const std::map<std::string, Tuning>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m)
    std::fprintf(f,
                 " \"%s\": {\"sap_wpe\": %d, \"sap_dom_rhs\": %d, \"sap_persist\": %d, \"dirac_threads\": %d, "
                 "\"coarse_spw\": %d}%s\n",
                 kv.first.c_str(), kv.second.sap_wpe, kv.second.sap_dom_rhs, kv.second.sap_persist,
                 kv.second.dirac_threads, kv.second.coarse_spw, ++i < m.size() ? "," : "");
  std::fprintf(f, "}\n");
  bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

extern "C" {

dd_status dd_setup(dd_gauge* g, const dd_mg_params* p, dd_mg** out) { return setup_common(g, p, nullptr, out); }

dd_status dd_setup_from_vectors(dd_gauge* g, const dd_mg_params* p, const double* tv_host, dd_mg** out) {
  if (!tv_host) return g ? dd_fail(g->ctx, DD_EINVAL, "null test vectors") : DD_EINVAL;
  return setup_common(g, p, tv_host, out);
}

dd_status dd_setup_update_mass(dd_mg* mg, double m0) {
  if (!mg) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  if (!std::isfinite(m0)) return dd_fail(mg->ctx, DD_EINVAL, "non-finite mass");
  if (mg->g->refcount != 1)
    return dd_fail(mg->ctx, DD_ESTATE, "another multigrid setup references this gauge field");
  DD_HIP(mg->ctx, hipSetDevice(mg->ctx->device));
  dd_status s = gauge_set_mass(mg->g, m0);
  if (s) return s;
  if ((s = build(mg, 0))) return s;
  return mg->l3 ? l3_galerkin(mg, 0) : DD_OK;   // D3 from the new D_c and the kept P2
}

dd_status dd_gauge_set_tuning(dd_gauge* g, const dd_tuning* t) {
  if (!g || !t) return DD_EINVAL;
  if ((t->sap_wpe != 2 && t->sap_wpe != 3) || (t->sap_dom_rhs != 0 && t->sap_dom_rhs != 2 && t->sap_dom_rhs != 4) ||
      (t->sap_persist != 0 && t->sap_persist != 1) ||
      (t->dirac_threads != 64 && t->dirac_threads != 128 && t->dirac_threads != 256) ||
      (t->coarse_spw != 2 && t->coarse_spw != 4 && t->coarse_spw != 8) || (t->coarse_half != 0 && t->coarse_half != 1) ||
      (t->coarse_basis_half != 0 && t->coarse_basis_half != 1) || (t->coarse_mfma_half != 0 && t->coarse_mfma_half != 1))
    return dd_fail(g->ctx, DD_EINVAL,
                   "tuning: sap_wpe 2|3, sap_dom_rhs 0|2|4, sap_persist 0|1, dirac_threads 64|128|256, coarse_spw 2|4|8, "
                   "coarse_half 0|1, "
                   "coarse_basis_half 0|1, coarse_mfma_half 0|1");
  g->tune.sap_wpe = t->sap_wpe;
  g->tune.sap_dom_rhs = t->sap_dom_rhs;
  g->tune.sap_persist = t->sap_persist;
  g->tune.dirac_threads = t->dirac_threads;
  g->tune.coarse_spw = t->coarse_spw;
  g->tune.coarse_half = t->coarse_half;
  g->tune.coarse_basis_half = t->coarse_basis_half;
  g->tune.coarse_mfma_half = t->coarse_mfma_half;
  return DD_OK;
}

dd_status dd_gauge_get_tuning(const dd_gauge* g, dd_tuning* t) {
  if (!g || !t) return DD_EINVAL;
  t->sap_wpe = g->tune.sap_wpe;
  t->sap_dom_rhs = g->tune.sap_dom_rhs;
  t->sap_persist = g->tune.sap_persist;
  t->dirac_threads = g->tune.dirac_threads;
  t->coarse_spw = g->tune.coarse_spw;
  t->coarse_half = g->tune.coarse_half;
  t->coarse_basis_half = g->tune.coarse_basis_half;
  t->coarse_mfma_half = g->tune.coarse_mfma_half;
  return DD_OK;
}

dd_status dd_autotune(dd_mg* mg, int nrhs, const char* cache_path, char* report, size_t report_cap) {
  if (!mg || nrhs < 1) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  if (mg->l3) return dd_fail(mg->ctx, DD_ESTATE, "tune before adding a third level");
  dd_gauge* g = mg->g;
  const GeomDev& G = g->geo;
  std::string key;
  {
    hipDeviceProp_t prop;
    DD_HIP(mg->ctx, hipGetDeviceProperties(&prop, mg->ctx->device));
    static const char* dn[4] = {"f64", "f32", "f16", "bf16"};
    char buf[256];
    // the coarse block type the caller chose is part of the key: the coarse launch shape is tuned for it
    std::snprintf(buf, sizeof(buf), "%s|L=%dx%dx%dx%d|b=%dx%dx%dx%d|n=%d|nrhs=%d|op=%s|inner=%s|cblk=%s",
                  prop.gcnArchName, G.L[0], G.L[1], G.L[2], G.L[3], G.b[0], G.b[1], G.b[2], G.b[3], mg->n, nrhs,
                  dn[op_dtype(mg)], dn[inner_vt(mg)],
                  (g->tune.coarse_half && mg->Dch) ? (g->tune.coarse_mfma_half ? "half-mfma" : "half") : "f32");
    key = buf;
  }
  std::map<std::string, Tuning> cache;
  if (cache_path) tune_cache_read(cache_path, cache);
  std::string rep = "key " + key + "\n";
  auto it = cache.find(key);
  // numerical choices of the caller (which coarse blocks, basis and products
  // the solve uses), not launch shapes: kept on a hit and on a miss
  const int coarse_half = g->tune.coarse_half, basis_half = g->tune.coarse_basis_half,
            mfma_half = g->tune.coarse_mfma_half;
  if (it != cache.end()) {
    g->tune = it->second;
    g->tune.coarse_half = coarse_half;
    g->tune.coarse_basis_half = basis_half;
    g->tune.coarse_mfma_half = mfma_half;
    rep += "cache hit\n";
  } else {
    dd_status s = ensure_ws(mg, nrhs, true);
    if (s) return s;
    Workspace* w = mg->ws;
    hipStream_t st = 0;
    hipEvent_t e0, e1;
    DD_HIP(mg->ctx, hipEventCreate(&e0));
    DD_HIP(mg->ctx, hipEventCreate(&e1));
    // median of 3 timed runs after one warm-up
    auto time_ms = [&](const std::function<void()>& f) {
      f();
      float t[3];
      for (int k = 0; k < 3; ++k) {
        (void)hipEventRecord(e0, st);
        f();
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&t[k], e0, e1);
      }
      std::sort(t, t + 3);
      return t[1];
    };
    char line[160];
    const dd_dtype od = op_dtype(mg), vt = inner_vt(mg);
    Tuning best = g->tune;
    // SAP: one sweep over scratch vectors of the workspace; the per-RHS layouts,
    // then (4^4 domains, half-precision operands) the domain-resident form
    if (od != DD_F64) {
      float bt = 1e30f;
      best.sap_dom_rhs = 0;
      for (int wpe : {2, 3}) {
        float t =
            time_ms([&] { launch_sap(G, od, g->ops[od], nrhs, 1, mg->p.sap_mr_iters, w->vin, w->xs, wpe, 0, 0, st); });
        std::snprintf(line, sizeof(line), "k_sap_colour sap_wpe=%d %.3f ms/sweep\n", wpe, t);
        rep += line;
        if (t < bt) bt = t, best.sap_wpe = wpe;
      }
      if (sap_dom_supported(G, od)) {
        for (int dr : {4, 2}) {
          float t =
              time_ms([&] { launch_sap(G, od, g->ops[od], nrhs, 1, mg->p.sap_mr_iters, w->vin, w->xs, 2, dr, 0, st); });
          std::snprintf(line, sizeof(line), "k_sap_dom sap_dom_rhs=%d %.3f ms/sweep\n", dr, t);
          rep += line;
          if (t < bt) bt = t, best.sap_dom_rhs = dr;
        }
        // the chosen domain form as one cooperative launch of all the smoother's sweeps
        best.sap_persist = 0;
        if (best.sap_dom_rhs) {
          const int sw = mg->p.sap_sweeps > 0 ? mg->p.sap_sweeps : 1;
          float t = time_ms([&] {
            launch_sap(G, od, g->ops[od], nrhs, sw, mg->p.sap_mr_iters, w->vin, w->xs, 2, best.sap_dom_rhs, 1, st);
          }) / sw;
          std::snprintf(line, sizeof(line), "k_sap_dom_persist sap_dom_rhs=%d %.3f ms/sweep\n", best.sap_dom_rhs, t);
          rep += line;
          if (t < bt) bt = t, best.sap_persist = 1;
        }
      }
    }
    // FP64 D apply of the outer solver
    {
      float bt = 1e30f;
      for (int th : {64, 128, 256}) {
        float t = time_ms([&] { launch_dirac(G, DD_F64, g->ops[DD_F64], nrhs, w->x64, w->zt64, st, th); });
        std::snprintf(line, sizeof(line), "k_dirac(f64) dirac_threads=%d %.3f ms\n", th, t);
        rep += line;
        if (t < bt) bt = t, best.dirac_threads = th;
      }
    }
    // coarse stencil on matrix cores, in the block type the caller chose
    if (vt == DD_F32) {
      float bt = 1e30f;
      for (int spw : {2, 4, 8}) {
        float t = time_ms([&] {
          CoarseOps c = coarse_ops(mg, vt);
          launch_coarse_mv(G, vt, mg->nc, c.Dc, c.Dinv, 0, nrhs, 0, G.Vc, 1.0, w->cb, 1.0, w->cb, 0.0, nullptr, w->cw,
                           st, spw, c.bt, c.hm);
        });
        std::snprintf(line, sizeof(line), "k_coarse_mfma coarse_spw=%d%s %.3f ms\n", spw,
                      g->tune.coarse_half && mg->Dch ? " (half blocks)" : "", t);
        rep += line;
        if (t < bt) bt = t, best.coarse_spw = spw;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    DD_HIP(mg->ctx, hipGetLastError());
    best.coarse_half = coarse_half;
    best.coarse_basis_half = basis_half;
    best.coarse_mfma_half = mfma_half;
    g->tune = best;
    cache[key] = best;
    if (cache_path && !tune_cache_write(cache_path, cache))
      rep += std::string("could not write ") + cache_path + "\n";
  }
  char line[128];
  std::snprintf(line, sizeof(line),
                "chosen sap_wpe=%d sap_dom_rhs=%d sap_persist=%d dirac_threads=%d coarse_spw=%d coarse_half=%d\n",
                g->tune.sap_wpe, g->tune.sap_dom_rhs, g->tune.sap_persist, g->tune.dirac_threads, g->tune.coarse_spw,
                g->tune.coarse_half);
  rep += line;
  if (report && report_cap) {
    std::strncpy(report, rep.c_str(), report_cap - 1);
    report[report_cap - 1] = 0;
  }
  return DD_OK;
}

dd_status dd_footprint_bytes(const dd_problem* prob, const dd_mg_params* p, int nrhs, dd_footprint* out) {
  if (!prob || !p || !out || nrhs < 1) return DD_EINVAL;
  long long V = 1, Vc = 1;
  for (int m = 0; m < 4; ++m) {
    const int L = prob->L[m], b = prob->block[m];
    if (b < 2 || (b & (b - 1)) || L < b || L % b || (L / b) % 2) return DD_ESHAPE;
    if (p->agg_block[m] != b || p->sap_block[m] != b) return DD_ESHAPE;
    V *= L;
    Vc *= L / b;
  }
  if (p->n_vec % 2 || !supported_nvec(p->n_vec)) return DD_ESHAPE;
  if (p->inner_dtype != DD_F64 && p->inner_dtype != DD_F32) return DD_EINVAL;
  if ((int)p->store_dtype < 0 || (int)p->store_dtype > 3) return DD_EINVAL;
  if ((p->inner_dtype == DD_F32) == (p->store_dtype == DD_F64)) return DD_EINVAL;
  if (p->coarse_restart < 1 || p->fgmres_restart < 1) return DD_EINVAL;
  const dd_dtype vt = p->inner_dtype == DD_F64 ? DD_F64 : DD_F32;
  const dd_dtype st = vt == DD_F64 ? DD_F64 : p->store_dtype;
  const long long n = p->n_vec, nc = 2 * n, nfine = 12 * V * n;
  const size_t fpair = 108ULL * V;   // links, clover and inverse: 36 complex pairs each per site
  // gauge: FP64 master, FP32 copy (also the source of half copies), half copy, block tables
  size_t gauge = 16 * fpair + 40ULL * Vc;
  if (st != DD_F64) gauge += 8 * fpair;
  if (st == DD_F16 || st == DD_BF16) gauge += 4 * fpair;
  // setup: P in FP64 and in the storage type, working vectors, D_c and inverses
  const size_t blocks = (size_t)nc * nc * (9 * Vc + Vc / 2);
  size_t setup = 16 * nfine + vector_pair_bytes(vt) * nfine + (st == DD_F64 ? 0 : storage_pair_bytes(st) * nfine) +
                 (16 + 8) * blocks;
  if (st == DD_F16 || st == DD_BF16) setup += 4 * blocks;
  // scratch while a setup runs: the V-cycle workspace for the n vectors, the
  // build's flag, then the FP32 staging of a half P or the Galerkin chunk
  const WsShape sh{V, Vc, Vc / 2, (int)nc, p->coarse_restart, p->fgmres_restart, vt};
  const long long vbytes = 12 * V * (long long)sizeof(double2);
  long long chunk = std::min<long long>((long long)((4ULL << 30) / (size_t)vbytes), nc);
  if (chunk >= 16 && chunk < nc) chunk -= chunk % 16;
  if (chunk < 1) chunk = 1;
  const size_t stage = (st == DD_F16 || st == DD_BF16) ? sizeof(float2) * (size_t)std::min<long long>(1LL << 27, nfine) : 0;
  const size_t build = std::max<size_t>(stage, (size_t)chunk * vbytes);
  const size_t upload = 16 * 36ULL * V;   // dd_gauge_create stages the canonical links
  out->gauge_bytes = gauge;
  out->setup_bytes = setup;
  out->scratch_bytes = std::max<size_t>(upload, ws_bytes(sh, (int)n, false) + sizeof(int) + build);
  out->workspace_bytes = ws_bytes(sh, nrhs, true);
  return DD_OK;
}

dd_status dd_mg_release_workspace(dd_mg* mg) {
  if (!mg) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  DD_HIP(mg->ctx, hipDeviceSynchronize());
  free_ws(mg);
  l3_free_ws(mg);
  return DD_OK;
}

dd_status dd_mg_set_graphs(dd_mg* mg, int mode) {
  if (!mg) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  if (mode < 0 || mode > 2) return dd_fail(mg->ctx, DD_EINVAL, "graph mode must be 0, 1 or 2");
  mg->graphs = mode;
  return DD_OK;
}

dd_status dd_mg_destroy(dd_mg* mg) {
  if (!mg) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  (void)hipDeviceSynchronize();
  mg_free(mg);
  return DD_OK;
}

size_t dd_coarse_vec_bytes(const dd_mg* mg, dd_dtype dt, int nrhs) {
  if (!mg || nrhs < 1) return 0;
  return vector_pair_bytes(dt) * (size_t)mg->g->geo.Vc * mg->nc * nrhs;
}

dd_status dd_pack_coarse(const dd_mg* mg, dd_dtype dt, int nrhs, const double* canon, void* packed, void* stream) {
  dd_status s = check_mg_vec((dd_mg*)mg, dt, nrhs, canon, packed);
  if (s) return s;
  launch_coarse_perm(mg->g->geo, dt, mg->nc, nrhs, 1, canon, packed, (hipStream_t)stream);
  DD_HIP(mg->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_unpack_coarse(const dd_mg* mg, dd_dtype dt, int nrhs, const void* packed, double* canon, void* stream) {
  dd_status s = check_mg_vec((dd_mg*)mg, dt, nrhs, packed, canon);
  if (s) return s;
  launch_coarse_perm(mg->g->geo, dt, mg->nc, nrhs, 0, packed, canon, (hipStream_t)stream);
  DD_HIP(mg->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_restrict(dd_mg* mg, dd_dtype dt, int nrhs, const void* fine, void* coarse, void* stream) {
  dd_status s = check_mg_vec(mg, dt, nrhs, fine, coarse);
  if (s) return s;
  const void* P = dt == DD_F64 ? (const void*)mg->P64 : (mg->vstore == DD_F64 ? (const void*)mg->P64 : mg->Pst);
  dd_dtype pdt = dt == DD_F64 ? DD_F64 : mg->vstore;
  launch_restrict(mg->g->geo, dt, pdt, mg->n, P, nrhs, fine, coarse, (hipStream_t)stream);
  DD_HIP(mg->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_prolong(dd_mg* mg, dd_dtype dt, int nrhs, const void* coarse, void* fine, void* stream) {
  dd_status s = check_mg_vec(mg, dt, nrhs, coarse, fine);
  if (s) return s;
  const void* P = dt == DD_F64 ? (const void*)mg->P64 : (mg->vstore == DD_F64 ? (const void*)mg->P64 : mg->Pst);
  dd_dtype pdt = dt == DD_F64 ? DD_F64 : mg->vstore;
  launch_prolong(mg->g->geo, dt, pdt, mg->n, P, nrhs, coarse, fine, (hipStream_t)stream);
  DD_HIP(mg->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_coarse_apply(dd_mg* mg, dd_dtype dt, int nrhs, const void* in, void* out, void* stream) {
  dd_status s = check_mg_vec(mg, dt, nrhs, in, out);
  if (s) return s;
  CoarseOps c = coarse_ops(mg, dt);
  launch_coarse_mv(mg->g->geo, dt, mg->nc, c.Dc, c.Dinv, 0, nrhs, 0, mg->g->geo.Vc, 1.0, in, 1.0, in, 0.0, nullptr,
                   out, (hipStream_t)stream, c.spw, c.bt, c.hm);
  DD_HIP(mg->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_coarse_solve(dd_mg* mg, dd_dtype dt, int nrhs, const void* in, void* out, int* iters, void* stream) {
  dd_status s = check_mg_vec(mg, dt, nrhs, in, out);
  if (s) return s;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  if (dt == DD_F64 && inner_vt(mg) != DD_F64)
    return dd_fail(mg->ctx, DD_EINVAL, "an FP32 setup's workspace holds no FP64 coarse basis: use DD_F32");
  if ((s = ensure_ws(mg, nrhs, false))) return s;
  return coarse_correction(mg, mg->ws, mg->graphs == 1, dt, nrhs, in, out, iters, (hipStream_t)stream);
}

dd_status dd_coarse_solve_noalloc(dd_mg* mg, dd_dtype dt, int nrhs, const void* in, void* out, int* iters,
                                  void* stream) {
  dd_status s = check_mg_vec(mg, dt, nrhs, in, out);
  if (s) return s;
  if (dt == DD_F64 && inner_vt(mg) != DD_F64)
    return dd_fail(mg->ctx, DD_EINVAL, "an FP32 setup's coarse solve runs in DD_F32");
  if (mg->l3) return dd_fail(mg->ctx, DD_ESTATE, "the allocation-free coarse solve is the two-level one: remove the third level");
  if (nrhs > kHostRhs)
    return dd_fail(mg->ctx, DD_EINVAL, "the allocation-free coarse solve takes at most " + std::to_string(kHostRhs) +
                                           " right-hand sides");
  if (!mg->ctx->scratch) return dd_fail(mg->ctx, DD_EDEVICE, "no static scratch address on this device");
  // the coarse part of the workspace, carved from the static scratch (a
  // workspace of the call's own dtype, so its basis holds that dtype)
  WsShape sh = ws_shape(mg);
  sh.vt = dt;
  Workspace w;
  w.nrhs = nrhs;
  w.arena.sizing = true;
  carve_ws(w, sh, nrhs, false, false);
  const size_t bytes = (w.arena.used + 255) & ~size_t(255);
  if (bytes > kStaticScratchBytes)
    return dd_fail(mg->ctx, DD_EBUDGET,
                   "the allocation-free coarse solve needs " + std::to_string(bytes) + " bytes of scratch; the static "
                   "array holds " + std::to_string(kStaticScratchBytes) + " (use fewer right-hand sides, a shorter "
                   "coarse restart, or dd_coarse_solve)");
  w.arena.base = (char*)mg->ctx->scratch;
  w.arena.cap = kStaticScratchBytes;
  w.arena.sizing = false;
  w.arena.used = 0;
  carve_ws(w, sh, nrhs, false, false);
  // host mirrors of the per-RHS flags on the stack (no pinned allocation)
  int hflags[2 * kHostRhs];
  double hvals[3 * kHostRhs];
  w.hflags = hflags;
  w.hvals = hvals;
  const hipStream_t st = (hipStream_t)stream;
  // the array keeps the last call's contents: start from zeros (finite basis entries)
  launch_zero(w.arena.base, bytes, st);
  w.cv_type = coarse_ops(mg, dt).basis;
  s = coarse_solve(mg, &w, false, dt, nrhs, in, out, iters, st);
  const hipError_t e = hipStreamSynchronize(st);   // the host mirrors live in this frame
  w.hflags = nullptr;
  w.hvals = nullptr;
  if (s) return s;
  if (e != hipSuccess) return dd_hip_check(mg->ctx, e, "allocation-free coarse solve");
  return DD_OK;
}

dd_status dd_precond_apply(dd_mg* mg, int nrhs, const void* in, void* out, void* stream) {
  dd_status s = check_mg_vec(mg, inner_vt(mg), nrhs, in, out);
  if (s) return s;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  if ((s = ensure_ws(mg, nrhs, false))) return s;
  return apply_M(mg, nrhs, in, out, nullptr, (hipStream_t)stream);
}

dd_status dd_export_coarse(const dd_mg* mg, double* dc_host) {
  if (!mg || !dc_host) return DD_EINVAL;
  const GeomDev& G = mg->g->geo;
  const int nc = mg->nc;
  std::vector<double2> buf((size_t)G.Vc * 9 * nc * nc);
  DD_HIP(mg->ctx, hipMemcpy(buf.data(), mg->Dc64, buf.size() * sizeof(double2), hipMemcpyDeviceToHost));
  int NB[4];
  for (int m = 0; m < 4; ++m) NB[m] = G.L[m] / G.b[m];
  for (int slot = 0; slot < G.Vc; ++slot) {
    int bc = mg->g->h_blk_coord[slot];
    int lex = (bc & 255) + NB[0] * (((bc >> 8) & 255) + NB[1] * (((bc >> 16) & 255) + NB[2] * ((bc >> 24) & 255)));
    for (int d = 0; d < 9; ++d)
      for (int col = 0; col < nc; ++col)
        for (int row = 0; row < nc; ++row) {
          double2 v = buf[(((size_t)slot * 9 + d) * nc + col) * nc + row];
          double* o = dc_host + ((((size_t)lex * 9 + d) * nc + row) * nc + col) * 2;
          o[0] = v.x;
          o[1] = v.y;
        }
  }
  return DD_OK;
}

dd_status dd_export_vectors(const dd_mg* mg, double* tv_host) {
  if (!mg || !tv_host) return DD_EINVAL;
  const GeomDev& G = mg->g->geo;
  size_t bytes = sizeof(double2) * 12ULL * G.V * mg->n;
  double2* tmp = nullptr;
  dd_status s = dd_alloc(mg->ctx, (void**)&tmp, bytes);
  if (s) return s;
  launch_unpack_fine(G, DD_F64, mg->n, mg->P64, tmp, 0);
  hipError_t e = hipMemcpy(tv_host, tmp, bytes, hipMemcpyDeviceToHost);
  dd_free(mg->ctx, tmp, bytes);
  if (e != hipSuccess) return dd_hip_check(mg->ctx, e, "export vectors");
  return DD_OK;
}

// ---------------------------------------------------------------------------
// outer flexible GMRES (FP64), right preconditioned by M
// ---------------------------------------------------------------------------
void dd_level3_params_default(dd_level3_params* p) {
  if (!p) return;
  p->n_vec2 = 24;
  p->setup_iters = 6;
  p->mr_steps = 6;
  p->kcycle_max_iters = 40;
  p->kcycle_fixed = 0;
  p->l3_restart = 60;
  p->l3_max_iters = 300;
  p->l3_fixed_iters = 0;
  p->kcycle_tol = 5e-2;
  p->l3_tol = 2e-1;
  p->seed = 0x13d3ULL;
}

dd_status dd_mg_add_level(dd_mg* mg, const dd_level3_params* p, const double* tv2_host) {
  if (!mg || !p) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  if (mg->l3) return dd_fail(mg->ctx, DD_ESTATE, "a third level is already attached");
  const int n2 = p->n_vec2;
  if (n2 != 6 && n2 != 8 && n2 != 12 && n2 != 16 && n2 != 20 && n2 != 24)
    return dd_fail(mg->ctx, DD_ESHAPE, "n_vec2 must be one of 6, 8, 12, 16, 20, 24");
  if (p->setup_iters < 0 || p->mr_steps < 0 || p->l3_fixed_iters < 0 || p->kcycle_max_iters < 1 ||
      p->kcycle_max_iters > 64 || p->l3_restart < 1 || p->l3_restart > 256 || p->l3_max_iters < 1 ||
      (p->kcycle_fixed != 0 && p->kcycle_fixed != 1) || !(p->kcycle_tol >= 0.0) || !(p->l3_tol >= 0.0))
    return dd_fail(mg->ctx, DD_EINVAL, "level-3 parameters out of range");
  const GeomDev& G = mg->g->geo;
  int NB[4];
  for (int m = 0; m < 4; ++m) {
    NB[m] = G.L[m] / G.b[m];
    if (NB[m] % 4) return dd_fail(mg->ctx, DD_ESHAPE, "every coarse-lattice extent must be a multiple of 4");
  }
  DD_HIP(mg->ctx, hipSetDevice(mg->ctx->device));
  Level3* L = new Level3();
  L->p = *p;
  L->n2 = n2;
  L->nc3 = 2 * n2;
  L->half = mg->Dch ? mg->vstore : DD_F64;
  for (int m = 0; m < 4; ++m) L->NB3[m] = NB[m] / 2;
  const int* N3 = L->NB3;
  L->Vc3 = N3[0] * N3[1] * N3[2] * N3[3];
  const int Vc3 = L->Vc3, Vch3 = Vc3 / 2;
  auto lex3 = [&](const int* c) { return c[0] + N3[0] * (c[1] + N3[1] * (c[2] + N3[2] * c[3])); };
  // level-3 slots as the block slots: even sites (coordinate sum even) first
  std::vector<int> slot3_of_lex(Vc3), coord3(4 * (size_t)Vc3);
  L->h_lex3.assign(Vc3, 0);
  for (int s3 = 0; s3 < Vc3; ++s3) {
    const int c = s3 / Vch3, k = s3 % Vch3, rest = (2 * k) / N3[0];
    int* x = &coord3[4 * (size_t)s3];
    x[1] = rest % N3[1];
    x[2] = (rest / N3[1]) % N3[2];
    x[3] = rest / (N3[1] * N3[2]);
    x[0] = (2 * k) % N3[0] + ((c + x[1] + x[2] + x[3]) & 1);
    L->h_lex3[s3] = lex3(x);
    slot3_of_lex[L->h_lex3[s3]] = s3;
  }
  std::vector<int> nbr3(8 * (size_t)Vc3);
  for (int s3 = 0; s3 < Vc3; ++s3)
    for (int mu = 0; mu < 4; ++mu)
      for (int sg = 0; sg < 2; ++sg) {
        int d[4] = {coord3[4 * s3], coord3[4 * s3 + 1], coord3[4 * s3 + 2], coord3[4 * s3 + 3]};
        d[mu] = (d[mu] + (sg == 0 ? 1 : -1) + N3[mu]) % N3[mu];
        nbr3[(sg * 4 + mu) * (size_t)Vc3 + s3] = slot3_of_lex[lex3(d)];
      }
  std::vector<int> slot_of(G.Vc), l3_of(G.Vc), loc_of(G.Vc);
  for (int x = 0; x < G.Vc; ++x) {
    const int bc = mg->g->h_blk_coord[x];
    const int c[4] = {bc & 255, (bc >> 8) & 255, (bc >> 16) & 255, (bc >> 24) & 255};
    const int h[4] = {c[0] / 2, c[1] / 2, c[2] / 2, c[3] / 2};
    const int l = (c[0] & 1) + 2 * ((c[1] & 1) + 2 * ((c[2] & 1) + 2 * (c[3] & 1)));
    const int X3 = slot3_of_lex[lex3(h)];
    slot_of[X3 * 16 + l] = x;
    l3_of[x] = X3;
    loc_of[x] = l;
  }
  Arena a;
  a.sizing = true;
  l3_carve(L, a, G.Vc, mg->n);
  L->bytes = a.used + 256;
  dd_status s = dd_alloc(mg->ctx, (void**)&L->base, L->bytes);
  if (s) {
    delete L;
    return s;
  }
  a.base = L->base;
  a.cap = L->bytes;
  a.sizing = false;
  a.used = 0;
  l3_carve(L, a, G.Vc, mg->n);
  mg->l3 = L;
  auto fail = [&](dd_status e) {
    (void)hipDeviceSynchronize();
    l3_free(mg);
    return e;
  };
  if (hipMemcpy(L->nbr3, nbr3.data(), sizeof(int) * nbr3.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(L->slot_of, slot_of.data(), sizeof(int) * G.Vc, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(L->l3_of, l3_of.data(), sizeof(int) * G.Vc, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(L->loc_of, loc_of.data(), sizeof(int) * G.Vc, hipMemcpyHostToDevice) != hipSuccess)
    return fail(dd_fail(mg->ctx, DD_EDEVICE, "level-3 table upload"));
  L->g3.Vc = Vc3;
  L->g3.Vch = Vch3;
  L->g3.blk_nbr = L->nbr3;
  // level-2 test vectors
  const hipStream_t st = 0;
  const long long ldc = (long long)G.Vc * mg->nc, nvec = ldc * n2;
  if (tv2_host) {
    double2* stage = nullptr;
    if ((s = dd_alloc(mg->ctx, (void**)&stage, sizeof(double2) * nvec))) return fail(s);
    hipError_t e = hipMemcpy(stage, tv2_host, sizeof(double2) * nvec, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      launch_coarse_perm(G, DD_F64, mg->nc, n2, 1, stage, L->tv2, st);
      e = hipStreamSynchronize(st);
    }
    dd_free(mg->ctx, stage, sizeof(double2) * nvec);
    if (e != hipSuccess) return fail(dd_hip_check(mg->ctx, e, "level-2 test vector upload"));
  } else {
    launch_gauss(p->seed, nvec, L->tv2, st);
    if (p->setup_iters > 0) {
      // inverse iteration with the two-level coarse solve, in the setup's inner dtype
      // (on a coarse-only workspace of its own: the setup's workspace may hold an outer solver's vectors)
      const dd_dtype vt = inner_vt(mg);
      const size_t vb = vector_pair_bytes(vt);
      Workspace* w = nullptr;
      const WsShape sh = ws_shape(mg);
      if ((s = alloc_ws(mg->ctx, n2, [&](Workspace& x) { carve_ws(x, sh, n2, false, false); }, &w))) return fail(s);
      char* buf = nullptr;
      if ((s = dd_alloc(mg->ctx, (void**)&buf, 2 * nvec * vb))) {
        destroy_ws(mg->ctx, w);
        return fail(s);
      }
      char *u = buf, *y = buf + nvec * vb;
      launch_vec_convert(DD_F64, vt, L->tv2, u, nvec, st);
      for (int k = 0; k < p->setup_iters && !s; ++k) {
        s = coarse_solve(mg, w, false, vt, n2, u, y, nullptr, st);
        norms2(w, vt, n2, ldc, ldc, y, w->ca.nrm2, st);
        launch_normalize(vt, n2, ldc, ldc, y, w->ca.nrm2, nullptr, nullptr, u, st, vt);
      }
      launch_vec_convert(vt, DD_F64, u, L->tv2, nvec, st);
      const hipError_t e = hipStreamSynchronize(st);
      dd_free(mg->ctx, buf, 2 * nvec * vb);
      destroy_ws(mg->ctx, w);
      if (s) return fail(s);
      if (e != hipSuccess) return fail(dd_hip_check(mg->ctx, e, "level-2 test vectors"));
    }
  }
  if ((s = l3_build(mg, st)) || (s = l3_galerkin(mg, st))) return fail(s);
  return DD_OK;
}

dd_status dd_mg_remove_level(dd_mg* mg) {
  if (!mg) return DD_EINVAL;
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  (void)hipDeviceSynchronize();
  l3_free(mg);
  return DD_OK;
}

dd_status dd_level3_shape(const dd_mg* mg, int32_t* vc3, int32_t* nc3) {
  if (!mg || !vc3 || !nc3) return DD_EINVAL;
  *vc3 = mg->l3 ? mg->l3->Vc3 : 0;
  *nc3 = mg->l3 ? mg->l3->nc3 : 0;
  return DD_OK;
}

dd_status dd_level3_last(const dd_mg* mg, int32_t* kcycle_steps, int32_t* l3_steps) {
  if (!mg || !kcycle_steps || !l3_steps) return DD_EINVAL;
  if (!mg->l3) return dd_fail(mg->ctx, DD_ESTATE, "no third level");
  *kcycle_steps = mg->l3->last_steps;
  *l3_steps = mg->l3->last_l3;
  return DD_OK;
}

dd_status dd_export_level3(const dd_mg* mg, double* tv2_host, double* p2_host, double* d3_host) {
  if (!mg) return DD_EINVAL;
  const Level3* L = mg->l3;
  if (!L) return dd_fail(mg->ctx, DD_ESTATE, "no third level");
  const GeomDev& G = mg->g->geo;
  const long long nvec = (long long)L->n2 * G.Vc * mg->nc, K = 16LL * mg->n, set = (long long)L->n2 * K;
  const int nc3 = L->nc3;
  if (tv2_host) {
    double2* stage = nullptr;
    dd_status s = dd_alloc(mg->ctx, (void**)&stage, sizeof(double2) * nvec);
    if (s) return s;
    launch_coarse_perm(G, DD_F64, mg->nc, L->n2, 0, L->tv2, stage, 0);
    const hipError_t e = hipMemcpy(tv2_host, stage, sizeof(double2) * nvec, hipMemcpyDeviceToHost);
    dd_free(mg->ctx, stage, sizeof(double2) * nvec);
    if (e != hipSuccess) return dd_hip_check(mg->ctx, e, "export level-2 vectors");
  }
  if (p2_host) {
    std::vector<double2> buf(nvec);
    DD_HIP(mg->ctx, hipMemcpy(buf.data(), L->P2_64, sizeof(double2) * nvec, hipMemcpyDeviceToHost));
    for (int X = 0; X < L->Vc3; ++X)
      for (long long e = 0; e < 2 * set; ++e) {
        const double2 v = buf[(size_t)X * 2 * set + e];
        double* o = p2_host + 2 * ((size_t)L->h_lex3[X] * 2 * set + e);
        o[0] = v.x;
        o[1] = v.y;
      }
  }
  if (d3_host) {
    std::vector<double2> buf((size_t)L->Vc3 * 9 * nc3 * nc3);
    DD_HIP(mg->ctx, hipMemcpy(buf.data(), L->D3_64, sizeof(double2) * buf.size(), hipMemcpyDeviceToHost));
    for (int X = 0; X < L->Vc3; ++X)
      for (int d = 0; d < 9; ++d)
        for (int col = 0; col < nc3; ++col)
          for (int row = 0; row < nc3; ++row) {
            const double2 v = buf[(((size_t)X * 9 + d) * nc3 + col) * nc3 + row];
            double* o = d3_host + 2 * ((((size_t)L->h_lex3[X] * 9 + d) * nc3 + row) * nc3 + col);
            o[0] = v.x;
            o[1] = v.y;
          }
  }
  return DD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// outer flexible GMRES (FP64), right preconditioned by M, as a sequence of
// restart cycles over slots: a right-hand side occupies a slot from the
// moment it is added until it is taken.  Adding a slot sets its residual to b
// (x = 0); one step is one restart cycle of the running slots followed by the
// true-residual check that decides which of them are done.  Slots are
// independent (per-RHS reductions and masks), so a right-hand side gets the
// same bits whether it starts alone, with others, or joins a running batch at
// a step boundary.
// ---------------------------------------------------------------------------
struct dd_solve_state {
  dd_mg* mg = nullptr;
  int cap = 0;
  double tol = 0.0;
  hipStream_t st = nullptr;
  std::vector<int> state;    // kSlotFree / kSlotRunning / kSlotDone
  std::vector<int> conv, iters, restarts;
  std::vector<double> bnorm, relres;
  int total_coarse = 0;
  double mb0 = 0.0, mf0 = 0.0;
  std::chrono::steady_clock::time_point t0;
};

enum { kSlotFree = 0, kSlotRunning = 1, kSlotDone = 2 };

// slot <- b: x = 0, r = b (a copy, as the first cycle of a solve from x = 0 takes it), |r|, tolerance
static dd_status solve_add(dd_solve_state* S, int slot, const double* b_canon) {
  dd_mg* mg = S->mg;
  Workspace* w = mg->ws;
  const GeomDev& G = mg->g->geo;
  const long long cnt = 12LL * G.V;
  hipStream_t st = S->st;
  double2* bs = w->b64 + (size_t)slot * cnt;
  double2* rs = w->w64 + (size_t)slot * cnt;
  launch_pack_fine(G, DD_F64, 1, (const double2*)b_canon, bs, st);
  DD_HIP(mg->ctx, hipMemsetAsync(w->x64 + (size_t)slot * cnt, 0, sizeof(double2) * cnt, st));
  DD_HIP(mg->ctx, hipMemcpyAsync(rs, bs, sizeof(double2) * cnt, hipMemcpyDeviceToDevice, st));
  norms2(w, DD_F64, 1, cnt, cnt, rs, w->fa.nrm2 + slot, st);
  double2 n2;
  DD_HIP(mg->ctx, hipMemcpyAsync(&n2, w->fa.nrm2 + slot, sizeof(double2), hipMemcpyDeviceToHost, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  const double bn = std::sqrt(n2.x);
  if (!std::isfinite(bn)) return dd_fail(mg->ctx, DD_ENAN, "non-finite right-hand side in slot " + std::to_string(slot));
  const double tl = S->tol * bn;
  DD_HIP(mg->ctx, hipMemcpyAsync(w->fa.tolabs + slot, &tl, sizeof(double), hipMemcpyHostToDevice, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  S->bnorm[slot] = bn;
  S->relres[slot] = bn == 0.0 ? 0.0 : 1.0;
  S->iters[slot] = S->restarts[slot] = 0;
  S->conv[slot] = S->relres[slot] <= S->tol ? 1 : 0;   // zero b: x = 0 is exact
  S->state[slot] = S->conv[slot] ? kSlotDone : kSlotRunning;
  return DD_OK;
}

// one restart cycle of the running slots, then their true-residual check
static dd_status solve_step(dd_solve_state* S) {
  dd_mg* mg = S->mg;
  Workspace* w = mg->ws;
  dd_gauge* g = mg->g;
  const GeomDev& G = g->geo;
  const long long cnt = 12LL * G.V;
  const dd_dtype vt = inner_vt(mg);
  const size_t vb = vector_pair_bytes(vt);
  Arnoldi& a = w->fa;
  const int m = a.m;
  hipStream_t st = S->st;
  dd_status s;
  int nhi = 0;   // slots [0, nhi) take part in the launches
  int longest = 0;
  for (int r = 0; r < S->cap; ++r)
    if (S->state[r] == kSlotRunning) {
      nhi = r + 1;
      longest = std::max(longest, S->iters[r]);
    }
  if (nhi == 0) return DD_OK;
  const long long fine = cnt * nhi;
  // the residuals r = b - D x of the running slots and their norms are in
  // w64 / nrm2 (from the last check, or from dd_solve_add)
  HostArr<int> fin(nhi, 1);
  for (int r = 0; r < nhi; ++r) fin[r] = S->state[r] == kSlotRunning ? 0 : 1;
  DD_HIP(mg->ctx, hipMemcpyAsync(a.finished, fin.p, sizeof(int) * nhi, hipMemcpyHostToDevice, st));
  launch_cycle_init(nhi, m, a.nrm2, a.tolabs, a.finished, a.gv, a.beta, a.active, a.kcyc, st);
  // with an FP32 preconditioner the normalisation also writes v_j rounded to FP32 (its input)
  void* vin32 = vt == DD_F64 ? nullptr : w->vin;
  const long long vs64 = fine, vsz = fine;   // basis strides (entries)
  launch_normalize(DD_F64, nhi, cnt, cnt, w->w64, nullptr, a.beta, a.active, w->V64, st, DD_F64, vin32);
  // the cycle ends at the restart length or where the longest-running slot reaches the iteration cap
  const int mm = mg->p.max_outer_iters - longest < m ? mg->p.max_outer_iters - longest : m;
  for (int j = 0; j < mm; ++j) {
    double2* Vj = w->V64 + (size_t)j * vs64;
    char* Zj = (char*)w->Z + (size_t)j * vsz * vb;
    // z_j = M v_j in the inner precision
    int ci = 0;
    if (vt == DD_F64) {
      if ((s = apply_M(mg, nhi, Vj, Zj, &ci, st))) return s;
      launch_dirac(G, DD_F64, g->ops[DD_F64], nhi, Zj, w->w64, st, g->tune.dirac_threads);
    } else {
      if ((s = apply_M(mg, nhi, w->vin, Zj, &ci, st))) return s;
      launch_dirac_f32_in(G, g->ops[DD_F64], nhi, (const float2*)Zj, w->w64, st, g->tune.dirac_threads);
    }
    S->total_coarse += ci;
    const int op = mg->p.outer_cgs_passes;
    cgs(w, a, DD_F64, nhi, cnt, cnt, w->V64, vs64, j + 1, w->w64, op, st, DD_F64);
    launch_arnoldi(nhi, m, j, a.h1, op == 2 ? a.h2 : nullptr, a.nrm2, a.H, a.cs, a.sn, a.gv, a.tolabs, a.active,
                   a.kcyc, a.est, a.hnext, st);
    if (j + 1 == mm) break;
    launch_normalize(DD_F64, nhi, cnt, cnt, w->w64, nullptr, a.hnext, a.active, w->V64 + (size_t)(j + 1) * vs64, st,
                     DD_F64, vin32);
    if (count_active(w, a.active, nhi, st) == 0) break;
  }
  launch_lsq(nhi, m, a.H, a.gv, a.kcyc, a.y, st);
  const int kmax = max_kcyc(w, a, nhi, st);   // also leaves kcyc in hflags[nhi..]
  launch_multi_axpy(vt, DD_F64, nhi, cnt, cnt, w->Z, kmax, vsz, a.y, m, 0, 1.0, w->x64, st);
  for (int r = 0; r < nhi; ++r)
    if (!fin[r]) {
      S->iters[r] += w->hflags[nhi + r];
      S->restarts[r] += 1;
    }
  // true residual r = b - D x with the FP64 operator
  launch_dirac(G, DD_F64, g->ops[DD_F64], nhi, w->x64, w->zt64, st, g->tune.dirac_threads);
  launch_sub(DD_F64, fine, w->b64, w->zt64, w->w64, st);
  norms2(w, DD_F64, nhi, cnt, cnt, w->w64, a.nrm2, st);
  HostArr<double2> n2(nhi);
  DD_HIP(mg->ctx, hipMemcpyAsync(n2.p, a.nrm2, sizeof(double2) * nhi, hipMemcpyDeviceToHost, st));
  DD_HIP(mg->ctx, hipStreamSynchronize(st));
  for (int r = 0; r < nhi; ++r) {
    if (fin[r]) continue;
    S->relres[r] = std::sqrt(n2[r].x) / S->bnorm[r];
    if (!std::isfinite(S->relres[r])) return dd_fail(mg->ctx, DD_ENAN, "breakdown: non-finite residual");
    if (S->relres[r] <= S->tol) {
      S->conv[r] = 1;
      S->state[r] = kSlotDone;
    } else if (S->iters[r] >= mg->p.max_outer_iters) {
      S->state[r] = kSlotDone;
    }
  }
  return DD_OK;
}

static void solve_info(const dd_solve_state* S, int r, dd_solve_info* info) {
  if (!info) return;
  double mb1, mf1;
  ktimer_model(&mb1, &mf1);
  info->outer_iters = S->iters[r];
  info->restarts = S->restarts[r];
  info->coarse_iters_total = S->total_coarse;
  info->converged = S->conv[r];
  info->true_relres = S->relres[r];
  info->t_setup_s = 0.0;
  info->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
  info->bytes_model = (int64_t)(mb1 - S->mb0);
  info->flops_model = (int64_t)(mf1 - S->mf0);
}

extern "C" {

dd_status dd_solve_begin(dd_mg* mg, int capacity, double tol, void* stream, dd_solve_state** out) {
  if (!mg || !out) return DD_EINVAL;
  *out = nullptr;
  if (capacity < 1 || !(tol > 0.0)) return dd_fail(mg->ctx, DD_EINVAL, "bad solve arguments");
  if (mg->live) return dd_fail(mg->ctx, DD_ESTATE, "a stepwise solve holds this multigrid's workspace");
  dd_status s = ensure_ws(mg, capacity, true);
  if (s) return s;
  dd_solve_state* S = new dd_solve_state();
  S->mg = mg;
  S->cap = capacity;
  S->tol = tol;
  S->st = (hipStream_t)stream;
  S->state.assign(capacity, kSlotFree);
  S->conv.assign(capacity, 0);
  S->iters.assign(capacity, 0);
  S->restarts.assign(capacity, 0);
  S->bnorm.assign(capacity, 0.0);
  S->relres.assign(capacity, 1.0);
  S->t0 = std::chrono::steady_clock::now();
  ktimer_model(&S->mb0, &S->mf0);
  if (whole_graph(mg)) launch_zero(mg->ws->citers, sizeof(int), S->st);   // coarse steps counted on the device
  mg->live = S;
  *out = S;
  return DD_OK;
}

dd_status dd_solve_add(dd_solve_state* S, int slot, const double* b_canon_dev) {
  if (!S) return DD_EINVAL;
  if (slot < 0 || slot >= S->cap || !b_canon_dev) return dd_fail(S->mg->ctx, DD_EINVAL, "bad slot or source");
  if (S->state[slot] != kSlotFree) return dd_fail(S->mg->ctx, DD_ESTATE, "slot " + std::to_string(slot) + " is in use");
  return solve_add(S, slot, b_canon_dev);
}

dd_status dd_solve_step(dd_solve_state* S, int32_t* slot_state) {
  if (!S) return DD_EINVAL;
  dd_status s = solve_step(S);
  if (slot_state)
    for (int r = 0; r < S->cap; ++r) slot_state[r] = S->state[r];
  return s;
}

dd_status dd_solve_take(dd_solve_state* S, int slot, double* x_canon_dev, dd_solve_info* info) {
  if (!S) return DD_EINVAL;
  if (slot < 0 || slot >= S->cap || !x_canon_dev) return dd_fail(S->mg->ctx, DD_EINVAL, "bad slot or output");
  if (S->state[slot] != kSlotDone) return dd_fail(S->mg->ctx, DD_ESTATE, "slot " + std::to_string(slot) + " is not done");
  dd_mg* mg = S->mg;
  const long long cnt = 12LL * mg->g->geo.V;
  launch_unpack_fine(mg->g->geo, DD_F64, 1, mg->ws->x64 + (size_t)slot * cnt, (double2*)x_canon_dev, S->st);
  if (whole_graph(mg))
    DD_HIP(mg->ctx, hipMemcpyAsync(&S->total_coarse, mg->ws->citers, sizeof(int), hipMemcpyDeviceToHost, S->st));
  DD_HIP(mg->ctx, hipStreamSynchronize(S->st));
  solve_info(S, slot, info);
  S->state[slot] = kSlotFree;
  return DD_OK;
}

dd_status dd_solve_end(dd_solve_state* S) {
  if (!S) return DD_EINVAL;
  if (S->mg->live == S) S->mg->live = nullptr;
  delete S;
  return DD_OK;
}

dd_status dd_solve(dd_mg* mg, int nrhs, const double* b_canon, double* x_canon, double tol, dd_solve_info* info,
                   void* stream) {
  if (!mg) return DD_EINVAL;
  if (!b_canon || !x_canon || nrhs < 1 || !(tol > 0.0)) return dd_fail(mg->ctx, DD_EINVAL, "bad solve arguments");
  dd_solve_state* S = nullptr;
  dd_status s = dd_solve_begin(mg, nrhs, tol, stream, &S);
  if (s) return s;
  const long long cnt = 12LL * mg->g->geo.V;
  for (int r = 0; r < nrhs && !s; ++r) s = solve_add(S, r, b_canon + 2 * (size_t)r * cnt);
  bool running = true;
  while (!s && running) {
    s = solve_step(S);
    running = false;
    for (int r = 0; r < nrhs; ++r) running = running || S->state[r] == kSlotRunning;
  }
  bool all = true;
  for (int r = 0; r < nrhs && !s; ++r) {
    all = all && S->conv[r];
    s = dd_solve_take(S, r, x_canon + 2 * (size_t)r * cnt, info ? info + r : nullptr);
  }
  dd_solve_end(S);
  if (s) return s;
  if (!all) return dd_fail(mg->ctx, DD_ENOCONV, "max_outer_iters reached before every right-hand side converged");
  return DD_OK;
}

}  // extern "C"

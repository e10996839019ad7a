// C ABI, part 1: contexts, errors, memory accounting, gauge fields, fine
// vectors and the operator apply.
#include <cmath>
#include <cstring>
#include <mutex>

#include "dd_internal.h"

// Static scratch for the allocation-free coarse solve (dd_coarse_solve_noalloc):
// every GPU the library runs on holds its own copy of this array until the
// process ends.  Host code never uses the array's name as a device address: the
// per-device address comes from hipGetSymbolAddress, taken once per device, with
// that device current, when the first context on it is created.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

// Device address of `device`'s scratch array (device current on entry).
static dd_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return DD_EDEVICE;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return DD_EDEVICE;
    }
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return DD_OK;
}

static const char* kStatus[] = {"DD_OK",    "DD_EINVAL", "DD_ESHAPE", "DD_ENOMEM", "DD_EBUDGET",
                                "DD_ENOCONV", "DD_ENAN", "DD_EDEVICE", "DD_ESTATE"};

// the last failure is kept per thread (and per context), so that threads driving
// different solvers on one context each read their own message
static thread_local const dd_ctx* t_err_ctx = nullptr;
static thread_local std::string t_err;

dd_status dd_fail(dd_ctx* ctx, dd_status s, const std::string& msg) {
  if (ctx) {
    t_err_ctx = ctx;
    t_err = std::string(kStatus[s]) + ": " + msg;
  }
  return s;
}

dd_status dd_hip_check(dd_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return dd_fail(ctx, DD_ENOMEM, std::string(what) + ": out of device memory");
  return dd_fail(ctx, DD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

dd_status dd_alloc(dd_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return DD_OK;
  {
    // reserve under the lock, allocate outside it
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->in_use + bytes > ctx->budget)
      return dd_fail(ctx, DD_EBUDGET, "allocation of " + std::to_string(bytes) + " bytes exceeds the HBM budget (" +
                                          std::to_string(ctx->in_use) + " of " + std::to_string(ctx->budget) +
                                          " in use)");
    ctx->in_use += bytes;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->in_use -= bytes;
    }
    return dd_hip_check(ctx, e, "hipMalloc");
  }
  return DD_OK;
}

void dd_free(dd_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->in_use -= bytes;
}

size_t ctx_in_use(dd_ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  return ctx->in_use;
}

extern "C" {

const char* dd_status_str(dd_status s) {
  if ((int)s < 0 || (int)s > 8) return "DD_UNKNOWN";
  return kStatus[s];
}

const char* dd_last_error(const dd_ctx* ctx) {
  if (!ctx) return "null context";
  return t_err_ctx == ctx ? t_err.c_str() : "";
}

size_t dd_ctx_bytes_in_use(const dd_ctx* ctx) { return ctx ? ctx_in_use(const_cast<dd_ctx*>(ctx)) : 0; }

dd_status dd_ctx_create(int device, size_t budget, dd_ctx** out) {
  if (!out) return DD_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DD_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return DD_EDEVICE;
  void* scr = nullptr;
  if (scratch_address(device, &scr) != DD_OK) scr = nullptr;   // only the allocation-free call needs it
  dd_ctx* c = new dd_ctx();
  c->device = device;
  c->budget = budget;
  c->in_use = 0;
  c->scratch = scr;
  *out = c;
  return DD_OK;
}

void dd_ctx_destroy(dd_ctx* ctx) { delete ctx; }

void dd_mg_params_default(dd_mg_params* p) {
  std::memset(p, 0, sizeof(*p));
  for (int m = 0; m < 4; ++m) p->agg_block[m] = p->sap_block[m] = 4;
  p->n_vec = 20;
  p->setup_iters = 4;
  p->init_sap_apps = 3;
  p->sap_sweeps = 4;
  p->sap_mr_iters = 4;
  p->coarse_restart = 60;
  p->coarse_max_iters = 300;
  p->coarse_fixed_iters = 0;
  p->fgmres_restart = 10;
  p->max_outer_iters = 200;
  p->coarse_tol = 5e-2;
  p->inner_dtype = DD_F32;
  p->store_dtype = DD_F32;
  p->seed = 1;
  p->coarse_cgs_passes = 1;
  p->outer_cgs_passes = 2;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// gauge fields
// ---------------------------------------------------------------------------
static bool is_pow2(int v) { return v >= 2 && (v & (v - 1)) == 0; }

static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

static dd_status build_geometry(dd_gauge* g) {
  const dd_problem& P = g->prob;
  GeomDev& G = g->geo;
  for (int m = 0; m < 4; ++m) {
    if (P.L[m] <= 0 || !is_pow2(P.block[m]) || P.L[m] % P.block[m])
      return dd_fail(g->ctx, DD_ESHAPE, "block edges must be powers of two >= 2 that divide L");
    if ((P.L[m] / P.block[m]) % 2)
      return dd_fail(g->ctx, DD_ESHAPE,
                     "every direction needs an even number of blocks (red-black SAP, coarse even-odd)");
    if (P.L[m] / P.block[m] > 255) return dd_fail(g->ctx, DD_ESHAPE, "more than 255 blocks in one direction");
    G.L[m] = P.L[m];
    G.b[m] = P.block[m];
    G.lb[m] = ilog2(P.block[m]);
  }
  if (P.bc_t != 1 && P.bc_t != -1) return dd_fail(g->ctx, DD_EINVAL, "bc_t must be +1 or -1");
  G.Bv = P.block[0] * P.block[1] * P.block[2] * P.block[3];
  if (G.Bv > 256) return dd_fail(g->ctx, DD_ESHAPE, "blocks hold at most 256 sites");
  G.lBv = ilog2(G.Bv);
  G.Bvh = G.Bv / 2;
  int NB[4];
  for (int m = 0; m < 4; ++m) NB[m] = P.L[m] / P.block[m];
  G.Vc = NB[0] * NB[1] * NB[2] * NB[3];
  G.Vch = G.Vc / 2;
  G.V = (long long)G.Vc * G.Bv;
  G.bc_t = (double)P.bc_t;
  // slot <-> block coordinates
  g->h_blk_coord.assign(G.Vc, 0);
  std::vector<int> slot_of_lex(G.Vc);
  for (int s = 0; s < G.Vc; ++s) {
    int c = s / G.Vch, k = s % G.Vch;
    int rest = (2 * k) / NB[0];
    int by = rest % NB[1], bz = (rest / NB[1]) % NB[2], bt = rest / (NB[1] * NB[2]);
    int delta = (c + by + bz + bt) & 1;
    int bx = (2 * k) % NB[0] + delta;
    g->h_blk_coord[s] = bx | (by << 8) | (bz << 16) | (bt << 24);
    slot_of_lex[bx + NB[0] * (by + NB[1] * (bz + NB[2] * bt))] = s;
  }
  g->h_blk_nbr.assign(8 * G.Vc, 0);
  for (int s = 0; s < G.Vc; ++s) {
    int bc = g->h_blk_coord[s];
    int c[4] = {bc & 255, (bc >> 8) & 255, (bc >> 16) & 255, (bc >> 24) & 255};
    for (int mu = 0; mu < 4; ++mu)
      for (int sg = 0; sg < 2; ++sg) {
        int d[4] = {c[0], c[1], c[2], c[3]};
        d[mu] += sg == 0 ? 1 : -1;
        bool wrap = d[mu] < 0 || d[mu] >= NB[mu];
        d[mu] = (d[mu] + NB[mu]) % NB[mu];
        int t = slot_of_lex[d[0] + NB[0] * (d[1] + NB[1] * (d[2] + NB[2] * d[3]))];
        if (wrap && mu == 3) t |= DD_WRAP_BIT;
        g->h_blk_nbr[(sg * 4 + mu) * G.Vc + s] = t;
      }
  }
  dd_status st;
  if ((st = dd_alloc(g->ctx, (void**)&g->d_blk_nbr, sizeof(int) * 8 * G.Vc))) return st;
  if ((st = dd_alloc(g->ctx, (void**)&g->d_blk_coord, sizeof(int) * G.Vc))) return st;
  if ((st = dd_alloc(g->ctx, (void**)&g->d_lex_slot, sizeof(int) * G.Vc))) return st;
  DD_HIP(g->ctx, hipMemcpy(g->d_blk_nbr, g->h_blk_nbr.data(), sizeof(int) * 8 * G.Vc, hipMemcpyHostToDevice));
  DD_HIP(g->ctx, hipMemcpy(g->d_blk_coord, g->h_blk_coord.data(), sizeof(int) * G.Vc, hipMemcpyHostToDevice));
  DD_HIP(g->ctx, hipMemcpy(g->d_lex_slot, slot_of_lex.data(), sizeof(int) * G.Vc, hipMemcpyHostToDevice));
  G.blk_nbr = g->d_blk_nbr;
  G.blk_coord = g->d_blk_coord;
  G.lex_slot = g->d_lex_slot;
  return DD_OK;
}

static size_t opset_bytes(const dd_gauge* g, dd_dtype dt) {
  return storage_pair_bytes(dt) * (size_t)g->geo.V * (36 + 36 + 36);
}

static void free_opset(dd_gauge* g, dd_dtype dt) {
  OpSet& o = g->ops[dt];
  size_t pb = storage_pair_bytes(dt) * (size_t)g->geo.V * 36;
  dd_free(g->ctx, o.links, pb);
  dd_free(g->ctx, o.clover, pb);
  dd_free(g->ctx, o.cinv, pb);
  o = OpSet();
}

// make the storage-dtype copies of links, clover and clover inverse from the FP64 master
dd_status ensure_opset(dd_gauge* g, dd_dtype dt) {
  OpSet& o = g->ops[dt];
  if (o.ready) return DD_OK;
  size_t pb = storage_pair_bytes(dt) * (size_t)g->geo.V * 36;
  dd_status st;
  // half-precision copies are rounded from the FP32 copy
  if ((dt == DD_F16 || dt == DD_BF16) && (st = ensure_opset(g, DD_F32))) return st;
  if ((st = dd_alloc(g->ctx, &o.links, pb)) || (st = dd_alloc(g->ctx, &o.clover, pb)) ||
      (st = dd_alloc(g->ctx, &o.cinv, pb))) {
    free_opset(g, dt);
    return st;
  }
  const OpSet& m = g->ops[DD_F64];
  const OpSet& f = g->ops[DD_F32];
  long long n = 36LL * g->geo.V;
  launch_convert_pairs(dt, (const double2*)m.links, (const float2*)f.links, o.links, n, 0);
  launch_convert_pairs(dt, (const double2*)m.clover, (const float2*)f.clover, o.clover, n, 0);
  launch_convert_pairs(dt, (const double2*)m.cinv, (const float2*)f.cinv, o.cinv, n, 0);
  DD_HIP(g->ctx, hipDeviceSynchronize());
  o.ready = true;
  return DD_OK;
}

// New bare mass on the same links: the clover term's diagonal is 4 + m0, so the
// FP64 clover and its inverse are rebuilt and every storage copy that exists is
// converted again (links are unchanged).
dd_status gauge_set_mass(dd_gauge* g, double m0) {
  OpSet& m = g->ops[DD_F64];
  g->prob.m0 = m0;
  launch_clover_build(g->geo, (const double2*)m.links, m0, g->prob.c_sw, (double2*)m.clover, (double2*)m.cinv, 0);
  const long long n = 36LL * g->geo.V;
  const dd_dtype order[3] = {DD_F32, DD_F16, DD_BF16};   // half copies are rounded from the FP32 copy
  for (dd_dtype dt : order) {
    OpSet& o = g->ops[dt];
    if (!o.ready) continue;
    const OpSet& f = g->ops[DD_F32];
    launch_convert_pairs(dt, (const double2*)m.clover, (const float2*)f.clover, o.clover, n, 0);
    launch_convert_pairs(dt, (const double2*)m.cinv, (const float2*)f.cinv, o.cinv, n, 0);
  }
  DD_HIP(g->ctx, hipDeviceSynchronize());
  return DD_OK;
}

static dd_status check_dtype(dd_ctx* ctx, dd_dtype dt) {
  if ((int)dt < 0 || (int)dt > 3) return dd_fail(ctx, DD_EINVAL, "unknown dtype");
  return DD_OK;
}

extern "C" {

dd_status dd_gauge_create(dd_ctx* ctx, const dd_problem* prob, const double* links_host, dd_gauge** out) {
  if (!ctx || !prob || !links_host || !out) return dd_fail(ctx, DD_EINVAL, "null argument");
  *out = nullptr;
  DD_HIP(ctx, hipSetDevice(ctx->device));
  dd_gauge* g = new dd_gauge();
  g->ctx = ctx;
  g->prob = *prob;
  dd_status st = build_geometry(g);
  if (st) {
    dd_gauge_destroy(g);
    return st;
  }
  OpSet& m = g->ops[DD_F64];
  size_t pb = 16 * (size_t)g->geo.V * 36;
  void* canon = nullptr;
  if ((st = dd_alloc(ctx, &m.links, pb)) || (st = dd_alloc(ctx, &m.clover, pb)) || (st = dd_alloc(ctx, &m.cinv, pb)) ||
      (st = dd_alloc(ctx, &canon, pb))) {
    dd_free(ctx, canon, pb);
    dd_gauge_destroy(g);
    return st;
  }
  hipError_t e = hipMemcpy(canon, links_host, pb, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_pack_links(g->geo, (const double2*)canon, (double2*)m.links, 0);
    launch_clover_build(g->geo, (const double2*)m.links, prob->m0, prob->c_sw, (double2*)m.clover, (double2*)m.cinv, 0);
    e = hipDeviceSynchronize();
  }
  dd_free(ctx, canon, pb);
  if (e != hipSuccess) {
    st = dd_hip_check(ctx, e, "gauge upload / clover build");
    dd_gauge_destroy(g);
    return st;
  }
  m.ready = true;
  *out = g;
  return DD_OK;
}

dd_status dd_gauge_set_mass(dd_gauge* g, double m0) {
  if (!g) return DD_EINVAL;
  if (!std::isfinite(m0)) return dd_fail(g->ctx, DD_EINVAL, "non-finite mass");
  if (g->refcount > 0)
    return dd_fail(g->ctx, DD_ESTATE, "gauge field is referenced by a multigrid setup; use dd_setup_update_mass");
  DD_HIP(g->ctx, hipSetDevice(g->ctx->device));
  return gauge_set_mass(g, m0);
}

dd_status dd_gauge_destroy(dd_gauge* g) {
  if (!g) return DD_EINVAL;
  if (g->refcount > 0) return dd_fail(g->ctx, DD_ESTATE, "gauge field is referenced by a multigrid setup");
  for (int d = 0; d < 4; ++d) free_opset(g, (dd_dtype)d);
  dd_free(g->ctx, g->d_blk_nbr, sizeof(int) * 8 * g->geo.Vc);
  dd_free(g->ctx, g->d_blk_coord, sizeof(int) * g->geo.Vc);
  dd_free(g->ctx, g->d_lex_slot, sizeof(int) * g->geo.Vc);
  delete g;
  return DD_OK;
}

size_t dd_fine_vec_bytes(const dd_gauge* g, dd_dtype dt, int nrhs) {
  if (!g || nrhs < 1) return 0;
  return vector_pair_bytes(dt) * 12 * (size_t)g->geo.V * nrhs;
}

dd_status dd_pack_fine(const dd_gauge* g, dd_dtype dt, int nrhs, const double* canon, void* packed, void* stream) {
  if (!g) return DD_EINVAL;
  dd_status st = check_dtype(g->ctx, dt);
  if (st) return st;
  if (!canon || !packed || nrhs < 1) return dd_fail(g->ctx, DD_EINVAL, "bad vector arguments");
  launch_pack_fine(g->geo, dt, nrhs, (const double2*)canon, packed, (hipStream_t)stream);
  DD_HIP(g->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_unpack_fine(const dd_gauge* g, dd_dtype dt, int nrhs, const void* packed, double* canon, void* stream) {
  if (!g) return DD_EINVAL;
  dd_status st = check_dtype(g->ctx, dt);
  if (st) return st;
  if (!canon || !packed || nrhs < 1) return dd_fail(g->ctx, DD_EINVAL, "bad vector arguments");
  launch_unpack_fine(g->geo, dt, nrhs, packed, (double2*)canon, (hipStream_t)stream);
  DD_HIP(g->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_dirac_apply(dd_gauge* g, dd_dtype dt, int nrhs, const void* in, void* out, void* stream) {
  if (!g) return DD_EINVAL;
  dd_status st = check_dtype(g->ctx, dt);
  if (st) return st;
  if (!in || !out || nrhs < 1) return dd_fail(g->ctx, DD_EINVAL, "bad vector arguments");
  if (in == out) return dd_fail(g->ctx, DD_EINVAL, "in and out must not alias");
  if ((st = ensure_opset(g, dt))) return st;
  launch_dirac(g->geo, dt, g->ops[dt], nrhs, in, out, (hipStream_t)stream, g->tune.dirac_threads);
  DD_HIP(g->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_sap_smooth(dd_gauge* g, const dd_mg_params* p, dd_dtype dt, int nrhs, const void* b, void* x,
                        void* stream) {
  if (!g) return DD_EINVAL;
  dd_status st = check_dtype(g->ctx, dt);
  if (st) return st;
  if (!p || !b || !x || nrhs < 1) return dd_fail(g->ctx, DD_EINVAL, "bad arguments");
  if (p->sap_sweeps < 0 || p->sap_mr_iters < 0) return dd_fail(g->ctx, DD_EINVAL, "negative SAP iteration counts");
  if (b == x) return dd_fail(g->ctx, DD_EINVAL, "b and x must not alias");
  if ((st = ensure_opset(g, dt))) return st;
  launch_sap(g->geo, dt, g->ops[dt], nrhs, p->sap_sweeps, p->sap_mr_iters, b, x, g->tune.sap_wpe, g->tune.sap_dom_rhs,
             g->tune.sap_persist, (hipStream_t)stream);
  DD_HIP(g->ctx, hipGetLastError());
  return DD_OK;
}

dd_status dd_export_maps(const dd_gauge* g, int32_t* agg_of_site, int32_t* local_of_site, int32_t* packed_index,
                         int8_t* color_of_block) {
  if (!g) return DD_EINVAL;
  const GeomDev& G = g->geo;
  const dd_problem& P = g->prob;
  int NB[4];
  for (int m = 0; m < 4; ++m) NB[m] = P.L[m] / P.block[m];
  for (long long x = 0; x < G.V; ++x) {
    long long r = x;
    int c[4];
    for (int m = 0; m < 4; ++m) {
      c[m] = (int)(r % P.L[m]);
      r /= P.L[m];
    }
    int bcrd[4], lc[4];
    for (int m = 0; m < 4; ++m) {
      bcrd[m] = c[m] / P.block[m];
      lc[m] = c[m] % P.block[m];
    }
    int agg = bcrd[0] + NB[0] * (bcrd[1] + NB[1] * (bcrd[2] + NB[2] * bcrd[3]));
    int loc = lc[0] + P.block[0] * (lc[1] + P.block[1] * (lc[2] + P.block[2] * lc[3]));
    if (agg_of_site) agg_of_site[x] = agg;
    if (local_of_site) local_of_site[x] = loc;
    if (packed_index) {
      int colour = (bcrd[0] + bcrd[1] + bcrd[2] + bcrd[3]) & 1;
      int slot = colour * G.Vch + agg / 2;
      int p = (c[0] + c[1] + c[2] + c[3]) & 1;
      packed_index[x] = slot * G.Bv + p * G.Bvh + loc / 2;
    }
  }
  if (color_of_block)
    for (int b = 0; b < G.Vc; ++b) {
      int bx = b % NB[0], by = (b / NB[0]) % NB[1], bz = (b / (NB[0] * NB[1])) % NB[2], bt = b / (NB[0] * NB[1] * NB[2]);
      color_of_block[b] = (int8_t)((bx + by + bz + bt) & 1);
    }
  return DD_OK;
}

dd_status dd_export_clover(const dd_gauge* g, double* clover_host, double* cinv_host) {
  if (!g) return DD_EINVAL;
  const GeomDev& G = g->geo;
  std::vector<double2> buf(36 * (size_t)G.V);
  std::vector<int32_t> pidx(G.V);
  dd_export_maps(g, nullptr, nullptr, pidx.data(), nullptr);
  for (int which = 0; which < 2; ++which) {
    double* dst = which ? cinv_host : clover_host;
    if (!dst) continue;
    const void* src = which ? g->ops[DD_F64].cinv : g->ops[DD_F64].clover;
    DD_HIP(g->ctx, hipMemcpy(buf.data(), src, buf.size() * sizeof(double2), hipMemcpyDeviceToHost));
    // packed [36 pairs][V] -> [lex][chirality][36 reals]: 6 diagonal reals, then 15 (re, im)
    for (long long x = 0; x < G.V; ++x) {
      long long I = pidx[x];
      for (int c = 0; c < 2; ++c) {
        double* o = dst + (x * 2 + c) * 36;
        for (int k = 0; k < 3; ++k) {
          double2 v = buf[(size_t)(18 * c + k) * G.V + I];
          o[2 * k] = v.x;
          o[2 * k + 1] = v.y;
        }
        for (int k = 0; k < 15; ++k) {
          double2 v = buf[(size_t)(18 * c + 3 + k) * G.V + I];
          o[6 + 2 * k] = v.x;
          o[7 + 2 * k] = v.y;
        }
      }
    }
  }
  return DD_OK;
}

dd_status dd_export_operands(dd_gauge* g, dd_dtype dt, void* links_host, void* clover_host) {
  if (!g) return DD_EINVAL;
  dd_status st = check_dtype(g->ctx, dt);
  if (st) return st;
  if ((st = ensure_opset(g, dt))) return st;
  size_t pb = storage_pair_bytes(dt) * (size_t)g->geo.V * 36;
  if (links_host) DD_HIP(g->ctx, hipMemcpy(links_host, g->ops[dt].links, pb, hipMemcpyDeviceToHost));
  if (clover_host) DD_HIP(g->ctx, hipMemcpy(clover_host, g->ops[dt].clover, pb, hipMemcpyDeviceToHost));
  return DD_OK;
}

}  // extern "C"

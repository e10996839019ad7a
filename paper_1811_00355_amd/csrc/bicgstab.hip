// The paper's comparison solver (Sec. 4, "baseline"): a nested mixed-precision
// BiCGstab whose single-precision level is preconditioned by SAP.  The paper
// does not spell out the outer iteration; here it is a defect correction with
// the FP64 operator (r = b - D x, x += e) around an FP32 BiCGstab on D e = r,
// right preconditioned by SAP (multiplicative red/black sweeps with the even-odd
// MR domain solver of the multigrid smoother), stopped at a relative residual.
// All right-hand sides advance together; a converged one gets zero update
// coefficients and stays as it is.  Scalars (rho, alpha, omega) are computed on
// the host from device dot products, three synchronisations per step.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "dd_internal.h"
#include "ktimer.h"

namespace {

// y_r = a_r x1_r + b_r x2_r + c_r x3_r for every right-hand side r (complex
// coefficients from device arrays of nrhs entries; a null array or vector
// drops its term).  Inputs may alias y: each element is read, then written, by
// one thread.
template <typename R, typename Tv>
__global__ void k_lincomb(int nrhs, long long cnt, const double2* __restrict__ ca, const Tv* x1,
                          const double2* __restrict__ cb, const Tv* x2, const double2* __restrict__ cc,
                          const Tv* x3, Tv* y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= cnt || r >= nrhs) return;
  const long long k = (long long)r * cnt + i;
  cx<R> acc = {(R)0, (R)0};
  if (ca && x1) cfma(acc, cx<R>{(R)ca[r].x, (R)ca[r].y}, ld<R, Tv>(x1 + k));
  if (cb && x2) cfma(acc, cx<R>{(R)cb[r].x, (R)cb[r].y}, ld<R, Tv>(x2 + k));
  if (cc && x3) cfma(acc, cx<R>{(R)cc[r].x, (R)cc[r].y}, ld<R, Tv>(x3 + k));
  st<Tv, R>(y + k, acc);
}

void lincomb(dd_dtype vt, int nrhs, long long cnt, const double2* ca, const void* x1, const double2* cb,
             const void* x2, const double2* cc, const void* x3, void* y, hipStream_t st) {
  dim3 grid((unsigned)((cnt + 255) / 256), nrhs);
  if (vt == DD_F64)
    k_lincomb<double, double2><<<grid, 256, 0, st>>>(nrhs, cnt, ca, (const double2*)x1, cb, (const double2*)x2, cc,
                                                      (const double2*)x3, (double2*)y);
  else
    k_lincomb<float, float2><<<grid, 256, 0, st>>>(nrhs, cnt, ca, (const float2*)x1, cb, (const float2*)x2, cc,
                                                    (const float2*)x3, (float2*)y);
}

typedef std::complex<double> C;

struct BiWs {
  dd_ctx* ctx = nullptr;
  std::vector<std::pair<void*, size_t>> bufs;
  void* take(size_t bytes, dd_status& s) {
    void* p = nullptr;
    if (!s) s = dd_alloc(ctx, &p, bytes);
    if (p) bufs.push_back({p, bytes});
    return p;
  }
  ~BiWs() {
    for (auto& b : bufs) dd_free(ctx, b.first, b.second);
  }
};

}  // namespace

extern "C" {

void dd_bicgstab_params_default(dd_bicgstab_params* p) {
  if (!p) return;
  p->sap_sweeps = 5;
  p->sap_mr_iters = 4;
  p->inner_max_iters = 500;
  p->max_outer_iters = 20;
  p->inner_tol = 1e-4;
  p->store_dtype = DD_F32;
  p->use_x0 = 0;
}

dd_status dd_solve_bicgstab(dd_gauge* g, const dd_bicgstab_params* p, int nrhs, const double* b_canon,
                            double* x_canon, double tol, dd_solve_info* info, void* stream) {
  if (!g || !p) return DD_EINVAL;
  dd_ctx* ctx = g->ctx;
  if (!b_canon || !x_canon || nrhs < 1 || !(tol > 0.0)) return dd_fail(ctx, DD_EINVAL, "bad solve arguments");
  if (p->sap_sweeps < 0 || p->sap_mr_iters < 0 || p->inner_max_iters < 1 || p->max_outer_iters < 1 ||
      !(p->inner_tol > 0.0 && p->inner_tol < 1.0))
    return dd_fail(ctx, DD_EINVAL, "bad BiCGstab parameters");
  const dd_dtype od = p->store_dtype;
  if (od != DD_F32 && od != DD_F16 && od != DD_BF16)
    return dd_fail(ctx, DD_EINVAL, "the FP32 inner level takes FP32, FP16 or BF16 operands");
  DD_HIP(ctx, hipSetDevice(ctx->device));
  const auto t0 = std::chrono::steady_clock::now();
  double mb0, mf0;
  ktimer_model(&mb0, &mf0);
  hipStream_t st = (hipStream_t)stream;
  dd_status s = ensure_opset(g, od);
  if (s) return s;
  const GeomDev& G = g->geo;
  const long long cnt = 12LL * G.V, fine = cnt * nrhs;
  const int nblk = dots_blocks(cnt, nrhs);

  BiWs ws;
  ws.ctx = ctx;
  s = DD_OK;
  double2* b64 = (double2*)ws.take(sizeof(double2) * fine, s);
  double2* x64 = (double2*)ws.take(sizeof(double2) * fine, s);
  double2* r64 = (double2*)ws.take(sizeof(double2) * fine, s);
  // FP32 inner vectors; (rt, r) and (t, s) adjacent so one launch gives both dots
  float2* rt = (float2*)ws.take(sizeof(float2) * fine * 2, s);
  float2* r = rt ? rt + fine : nullptr;
  float2* t = (float2*)ws.take(sizeof(float2) * fine * 2, s);
  float2* sv = t ? t + fine : nullptr;
  float2* e = (float2*)ws.take(sizeof(float2) * fine, s);
  float2* pv = (float2*)ws.take(sizeof(float2) * fine, s);
  float2* v = (float2*)ws.take(sizeof(float2) * fine, s);
  float2* mp = (float2*)ws.take(sizeof(float2) * fine, s);
  float2* ms = (float2*)ws.take(sizeof(float2) * fine, s);
  double* partial = (double*)ws.take(sizeof(double) * nrhs * 16 * nblk * 2, s);
  double2* dots = (double2*)ws.take(sizeof(double2) * nrhs * 2, s);
  double2* coef = (double2*)ws.take(sizeof(double2) * nrhs * 3, s);
  if (s) return s;
  double2 *ca = coef, *cb = coef + nrhs, *cc = coef + 2 * nrhs;

  std::vector<double2> hd(2 * nrhs), hc(3 * nrhs);
  auto read_dots = [&](int k) -> dd_status {
    DD_HIP(ctx, hipMemcpyAsync(hd.data(), dots, sizeof(double2) * nrhs * k, hipMemcpyDeviceToHost, st));
    DD_HIP(ctx, hipStreamSynchronize(st));
    return DD_OK;
  };
  auto put_coef = [&]() -> dd_status {
    DD_HIP(ctx, hipMemcpyAsync(coef, hc.data(), sizeof(double2) * nrhs * 3, hipMemcpyHostToDevice, st));
    return DD_OK;
  };
  auto set = [&](int which, int rr, C z) { hc[which * nrhs + rr] = make_double2(z.real(), z.imag()); };
  // M applied from zero: out = SAP(in)
  auto precond = [&](const float2* in, float2* out) {
    launch_zero(out, sizeof(float2) * fine, st);
    launch_sap(G, od, g->ops[od], nrhs, p->sap_sweeps, p->sap_mr_iters, in, out, g->tune.sap_wpe, g->tune.sap_dom_rhs,
               g->tune.sap_persist, st);
  };
  auto apply_D = [&](const float2* in, float2* out) {
    launch_dirac(G, od, g->ops[od], nrhs, in, out, st, g->tune.dirac_threads);
  };

  launch_pack_fine(G, DD_F64, nrhs, (const double2*)b_canon, b64, st);
  if (p->use_x0) launch_pack_fine(G, DD_F64, nrhs, (const double2*)x_canon, x64, st);
  else launch_zero(x64, sizeof(double2) * fine, st);
  launch_dots(DD_F64, DD_F64, nrhs, cnt, cnt, b64, 1, 0, b64, partial, nblk, dots, 1, 0, st);
  if ((s = read_dots(1))) return s;
  std::vector<double> bnorm(nrhs), relres(nrhs, 1.0);
  std::vector<int> fin(nrhs, 0);
  for (int q = 0; q < nrhs; ++q) {
    bnorm[q] = std::sqrt(hd[q].x);
    if (!std::isfinite(bnorm[q])) return dd_fail(ctx, DD_ENAN, "non-finite right-hand side " + std::to_string(q));
    if (bnorm[q] == 0.0) fin[q] = 1, relres[q] = 0.0;
  }
  int outer = 0, inner_total = 0;
  while (true) {
    // r64 = b - D x (FP64 operator); without a starting guess x = 0 on the first pass
    if (outer == 0 && !p->use_x0) {
      DD_HIP(ctx, hipMemcpyAsync(r64, b64, sizeof(double2) * fine, hipMemcpyDeviceToDevice, st));
    } else {
      launch_dirac(G, DD_F64, g->ops[DD_F64], nrhs, x64, r64, st, g->tune.dirac_threads);
      launch_sub(DD_F64, fine, b64, r64, r64, st);
    }
    launch_dots(DD_F64, DD_F64, nrhs, cnt, cnt, r64, 1, 0, r64, partial, nblk, dots, 1, 0, st);
    if ((s = read_dots(1))) return s;
    int nfin = 0;
    bool grew = false;
    for (int q = 0; q < nrhs; ++q) {
      const double before = relres[q];
      if (bnorm[q] > 0.0) relres[q] = std::sqrt(hd[q].x) / bnorm[q];
      if (!std::isfinite(relres[q])) return dd_fail(ctx, DD_ENAN, "breakdown: non-finite residual");
      if (relres[q] <= tol) fin[q] = 1;
      if (outer > 0 && !fin[q] && relres[q] > before) grew = true;   // the inner solve made it worse
      nfin += fin[q];
    }
    if (nfin == nrhs || outer >= p->max_outer_iters || grew) break;
    ++outer;
    // inner right-hand side: r in FP32, zero for finished right-hand sides
    launch_vec_convert(DD_F64, DD_F32, r64, r, fine, st);
    for (int q = 0; q < nrhs; ++q) set(0, q, fin[q] ? C(0.0) : C(1.0)), set(1, q, 0.0), set(2, q, 0.0);
    if ((s = put_coef())) return s;
    lincomb(DD_F32, nrhs, cnt, ca, r, nullptr, nullptr, nullptr, nullptr, r, st);
    DD_HIP(ctx, hipMemcpyAsync(rt, r, sizeof(float2) * fine, hipMemcpyDeviceToDevice, st));
    launch_zero(e, sizeof(float2) * fine, st);
    launch_zero(pv, sizeof(float2) * fine, st);
    launch_zero(v, sizeof(float2) * fine, st);
    std::vector<C> rho(nrhs, 1.0), alpha(nrhs, 1.0), omega(nrhs, 1.0);
    std::vector<double> nb0(nrhs, 0.0);
    std::vector<int> act(nrhs, 0);
    for (int it = 0; it <= p->inner_max_iters; ++it) {
      // (rt, r) and (r, r)
      launch_dots(DD_F32, DD_F32, nrhs, cnt, cnt, rt, 2, fine, r, partial, nblk, dots, 2, 0, st);
      if ((s = read_dots(2))) return s;
      int nact = 0;
      for (int q = 0; q < nrhs; ++q) {
        const double rn = std::sqrt(hd[2 * q + 1].x);
        if (it == 0) nb0[q] = rn;
        act[q] = it < p->inner_max_iters && rn > p->inner_tol * nb0[q] && nb0[q] > 0.0;
        nact += act[q];
      }
      if (nact == 0) break;
      ++inner_total;
      // p = r + beta (p - omega v)
      std::vector<C> rho_new(nrhs);
      for (int q = 0; q < nrhs; ++q) {
        rho_new[q] = C(hd[2 * q].x, hd[2 * q].y);
        if (act[q]) {
          const C beta = (rho_new[q] / rho[q]) * (alpha[q] / omega[q]);
          set(0, q, beta), set(1, q, 1.0), set(2, q, -beta * omega[q]);
          rho[q] = rho_new[q];
        } else {
          set(0, q, 1.0), set(1, q, 0.0), set(2, q, 0.0);
        }
      }
      if ((s = put_coef())) return s;
      lincomb(DD_F32, nrhs, cnt, ca, pv, cb, r, cc, v, pv, st);
      precond(pv, mp);
      apply_D(mp, v);
      // alpha = rho / (rt, v)
      launch_dots(DD_F32, DD_F32, nrhs, cnt, cnt, rt, 1, 0, v, partial, nblk, dots, 1, 0, st);
      if ((s = read_dots(1))) return s;
      for (int q = 0; q < nrhs; ++q) {
        alpha[q] = act[q] ? rho[q] / C(hd[q].x, hd[q].y) : C(0.0);
        set(0, q, 1.0), set(1, q, -alpha[q]), set(2, q, 0.0);
      }
      if ((s = put_coef())) return s;
      lincomb(DD_F32, nrhs, cnt, ca, r, cb, v, nullptr, nullptr, sv, st);   // s = r - alpha v
      precond(sv, ms);
      apply_D(ms, t);
      // omega = (t, s) / (t, t): V = {t, s} against w = t gives (t, t) and conj((t, s))
      launch_dots(DD_F32, DD_F32, nrhs, cnt, cnt, t, 2, fine, t, partial, nblk, dots, 2, 0, st);
      if ((s = read_dots(2))) return s;
      for (int q = 0; q < nrhs; ++q) {
        const double tt = hd[2 * q].x;
        omega[q] = (act[q] && tt > 0.0) ? std::conj(C(hd[2 * q + 1].x, hd[2 * q + 1].y)) / tt : C(0.0);
        set(0, q, 1.0), set(1, q, alpha[q]), set(2, q, omega[q]);
      }
      if ((s = put_coef())) return s;
      lincomb(DD_F32, nrhs, cnt, ca, e, cb, mp, cc, ms, e, st);          // e += alpha M p + omega M s
      for (int q = 0; q < nrhs; ++q) set(0, q, 1.0), set(1, q, -omega[q]), set(2, q, 0.0);
      if ((s = put_coef())) return s;
      lincomb(DD_F32, nrhs, cnt, ca, sv, cb, t, nullptr, nullptr, r, st);  // r = s - omega t
      // a right-hand side whose omega vanished cannot continue
      for (int q = 0; q < nrhs; ++q)
        if (act[q] && omega[q] == C(0.0)) omega[q] = 1.0, rho[q] = 1.0;
    }
    // x += e (the FP32 correction, widened)
    launch_vec_convert(DD_F32, DD_F64, e, r64, fine, st);
    launch_add(DD_F64, fine, r64, x64, st);
  }
  launch_unpack_fine(G, DD_F64, nrhs, x64, (double2*)x_canon, st);
  DD_HIP(ctx, hipStreamSynchronize(st));
  const double tsolve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  double mb1, mf1;
  ktimer_model(&mb1, &mf1);
  bool all = true;
  for (int q = 0; q < nrhs; ++q) {
    all = all && fin[q];
    if (info) {
      info[q].outer_iters = outer;
      info[q].restarts = 0;
      info[q].coarse_iters_total = inner_total;   // inner BiCGstab steps (all right-hand sides together)
      info[q].converged = fin[q];
      info[q].true_relres = relres[q];
      info[q].t_setup_s = 0.0;
      info[q].t_solve_s = tsolve;
      info[q].bytes_model = (int64_t)(mb1 - mb0);
      info[q].flops_model = (int64_t)(mf1 - mf0);
    }
  }
  if (!all)
    return dd_fail(ctx, DD_ENOCONV,
                   "defect correction stopped (max_outer_iters, or a step increased the residual) before every "
                   "right-hand side converged");
  return DD_OK;
}

}  // extern "C"

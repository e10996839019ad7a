// SAP smoother (Sec. 2): multiplicative Schwarz over the red and black
// domains.  One launch per colour; one workgroup per (domain, right-hand side).
//
// For every domain B of the colour:
//   r_B   = b - D x on the sites of B      (full operator: the halo of x comes
//                                           from the neighbouring domains of the
//                                           other colour, which this launch
//                                           does not modify)
//   rhs_e = r_e - H_eo A_oo^-1 r_o          (H = hopping term kept inside B)
//   MR on S = A_ee - H_eo A_oo^-1 H_oe from e_e = 0, a fixed number of steps
//   e_o   = A_oo^-1 (r_o - H_oe e_e)
//   x_B  += e
// Recomputing r_B from x at the start of every domain solve is the same
// multiplicative iteration as carrying a global residual, without storing one.
//
// Thread j of a workgroup owns the even site j and the odd site j of the
// domain; the half-lattice vectors exchanged between the even and odd phases
// live in LDS.  Domains hold at most 256 sites.
#include "dslash.h"
#include "ktimer.h"

namespace {

constexpr int kMaxBvh = 128;

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum of (a, b, c) over the workgroup; deterministic order
template <typename R>
__device__ __forceinline__ void block_sum3(R& a, R& b, R& c, R* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[3 * w] = a;
    red[3 * w + 1] = b;
    red[3 * w + 2] = c;
  }
  __syncthreads();
  a = b = c = (R)0;
  for (int i = 0; i < nw; ++i) {
    a += red[3 * i];
    b += red[3 * i + 1];
    c += red[3 * i + 2];
  }
}

// Two layouts of the same arithmetic (bit-identical results), picked by WPE,
// the waves per SIMD the register allocation must allow:
//  WPE 2: the correction e_e lives in registers; the odd residual r_o and the
//         even and odd exchange vectors have LDS buffers of their own (36 KB
//         in FP32, which also limits a CU to 2 waves per SIMD).
//  WPE 3: e_e lives in LDS, one exchange buffer serves both phases (two more
//         barriers per MR step) and r_o is recomputed for the reconstruction
//         instead of being kept (24 KB, 3 waves per SIMD).
template <typename R, typename S, typename Tv, int WPE>
__global__ void __launch_bounds__(kMaxBvh) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_sap_colour(GeomDev g, const S* __restrict__ links, const S* __restrict__ clov, const S* __restrict__ cinv, int nrhs,
             int colour, int mr_iters, const Tv* __restrict__ bvec, Tv* __restrict__ xvec) {
  constexpr bool kLean = WPE >= 3;
  constexpr int kE = kLean ? kMaxBvh : 1;    // LDS slots of e_e (lean layout)
  constexpr int kX = kLean ? 1 : kMaxBvh;    // second exchange buffer and r_o (register layout)
  __shared__ cx<R> sh[12][kMaxBvh];    // even-phase output read by the odd phase (and, lean: both ways)
  __shared__ cx<R> sh_o[12][kX];       // odd-phase output read by the even phase
  __shared__ cx<R> sh_r[12][kX];       // odd residual r_o
  __shared__ cx<R> se_acc[12][kE];     // e_e
  __shared__ R red[3 * (kMaxBvh / 64 + 1)];
  cx<R>(*sh_odd)[kMaxBvh] = kLean ? sh : (cx<R>(*)[kMaxBvh])sh_o;

  // domains of one colour are numbered in lexicographic block order; each XCD
  // takes a contiguous range of them, so the 8 domains around a block of the
  // other colour (whose x is their halo) run on one L2
  int tile, r;
  xcd_range_tile(g.Vch, nrhs, tile, r);
  if (tile >= g.Vch) return;
  const int slot = colour * g.Vch + tile;
  const int j = threadIdx.x;
  const bool act = j < g.Bvh;
  const long long V = g.V;
  const Tv* b = bvec + (long long)r * 12 * V;
  Tv* x = xvec + (long long)r * 12 * V;
  const long long Ie = ((long long)slot << g.lBv) + j;
  const long long Io = Ie + g.Bvh;

  auto fetch_x = [&](long long J, bool, cx<R>* p) { load_spinor<R, Tv>(x, V, J, p); };
  auto fetch_sh = [&](long long J, bool, cx<R>* p) {
    int jj = (int)(J & (g.Bvh - 1));
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = sh[c][jj];
  };
  auto fetch_odd = [&](long long J, bool, cx<R>* p) {
    int jj = (int)(J & (g.Bvh - 1));
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = sh_odd[c][jj];
  };
  auto fetch_e = [&](long long J, bool, cx<R>* p) {
    int jj = (int)(J & (g.Bvh - 1));
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = se_acc[c][jj];
  };

  cx<R> rho[12], t[12], e[kLean ? 1 : 12];
  SiteLoc se, so;
  if (act) {
    se = decode_site(g, Ie);
    so = decode_site(g, Io);
    // odd site: r_o = b - D x (kept in the register layout), A_oo^-1 r_o to the exchange buffer
    load_spinor<R, Tv>(x, V, Io, rho);
    clover_mul<R, S, false>(clov, V, Io, rho, t);
    load_spinor<R, Tv>(b, V, Io, rho);
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = rho[c] - t[c];
    hop_all<R, S>(g, links, so, Io, false, fetch_x, rho, (R)-1);
    if (!kLean) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sh_r[c][j] = rho[c];
    }
    clover_mul<R, S, false>(cinv, V, Io, rho, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) sh_odd[c][j] = t[c];
    // even site: r_e = b - D x
    load_spinor<R, Tv>(x, V, Ie, rho);
    clover_mul<R, S, false>(clov, V, Ie, rho, t);
    load_spinor<R, Tv>(b, V, Ie, rho);
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = rho[c] - t[c];
    hop_all<R, S>(g, links, se, Ie, false, fetch_x, rho, (R)-1);
  }
  __syncthreads();
  if (act) {
    // rhs_e = r_e - H_eo A_oo^-1 r_o ; MR starts from e_e = 0 with rho = rhs_e
    hop_all<R, S>(g, links, se, Ie, true, fetch_odd, rho, (R)-1);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      if (kLean) se_acc[c][j] = {(R)0, (R)0};
      else e[c] = {(R)0, (R)0};
    }
  }
#pragma unroll 1
  for (int k = 0; k < mr_iters; ++k) {
    if (kLean) __syncthreads();   // every read of the shared buffer is done before it is rewritten
    if (act) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sh[c][j] = rho[c];
    }
    __syncthreads();
    cx<R> u[12];
    if (act) {
      // odd: u = A_oo^-1 H_oe rho
#pragma unroll
      for (int c = 0; c < 12; ++c) t[c] = {(R)0, (R)0};
      hop_all<R, S>(g, links, so, Io, true, fetch_sh, t);
      clover_mul<R, S, false>(cinv, V, Io, t, u);
    }
    if (kLean) __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sh_odd[c][j] = u[c];
    }
    __syncthreads();
    R pr_re = 0, pr_im = 0, pp = 0;
    if (act) {
      // even: p = A_ee rho - H_eo u   (kept in t)
      clover_mul<R, S, false>(clov, V, Ie, rho, t);
      hop_all<R, S>(g, links, se, Ie, true, fetch_odd, t, (R)-1);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        cx<R> q = cmul_conj(t[c], rho[c]);   // conj(p) rho
        pr_re += q.re;
        pr_im += q.im;
        pp += t[c].re * t[c].re + t[c].im * t[c].im;
      }
    }
    block_sum3(pr_re, pr_im, pp, red);   // its barriers also close the reads of the exchange buffers
    if (act) {
      cx<R> alpha = {(R)0, (R)0};
      if (pp > (R)0) alpha = {pr_re / pp, pr_im / pp};
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        if (kLean) {
          cx<R> ev = se_acc[c][j];
          cfma(ev, alpha, rho[c]);
          se_acc[c][j] = ev;
        } else {
          cfma(e[c], alpha, rho[c]);
        }
        rho[c] = rho[c] - alpha * t[c];
      }
    }
  }
  if (kLean) {
    if (act) {
      // r_o again (x is still the old x everywhere it is read)
      load_spinor<R, Tv>(x, V, Io, t);
      clover_mul<R, S, false>(clov, V, Io, t, rho);
      load_spinor<R, Tv>(b, V, Io, t);
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = t[c] - rho[c];
      hop_all<R, S>(g, links, so, Io, false, fetch_x, rho, (R)-1);
    }
    __syncthreads();   // all reads of the old x are done before x is written
  } else {
    if (act) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sh[c][j] = e[c];
    }
    __syncthreads();
  }
  if (act) {
    // x_e += e_e
    load_spinor<R, Tv>(x, V, Ie, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) t[c] = t[c] + (kLean ? se_acc[c][j] : e[c]);
    store_spinor<R, Tv>(x, V, Ie, t);
    // e_o = A_oo^-1 (r_o - H_oe e_e);  x_o += e_o
    if (kLean) {
      hop_all<R, S>(g, links, so, Io, true, fetch_e, rho, (R)-1);
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = sh_r[c][j];
      hop_all<R, S>(g, links, so, Io, true, fetch_sh, rho, (R)-1);
    }
    clover_mul<R, S, false>(cinv, V, Io, rho, t);
    load_spinor<R, Tv>(x, V, Io, rho);
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = rho[c] + t[c];
    store_spinor<R, Tv>(x, V, Io, rho);
  }
}

template <typename R, typename S, typename Tv, int WPE>
void run(const GeomDev& g, const OpSet& ops, int nrhs, int sweeps, int mr, const void* b, void* x, hipStream_t st) {
  int threads = ((g.Bvh + 63) / 64) * 64;
  unsigned nb = xcd_grid(g.Vch, nrhs);
  // per launch (one colour = half the sites): links, clover and odd-site inverse
  // once, b and x read and x written per RHS; useful flops per site and RHS
  // (k + 2.5) operator applies of 1850 flops: the residual, k MR steps with
  // their Schur products, and the source projection and odd reconstruction
  const double half = 0.5 * (double)g.V;
  const double bytes = half * (90.0 * sizeof(S) + 36.0 * sizeof(Tv) * nrhs);
  const double flops = half * nrhs * (mr + 2.5) * 1850.0;
  for (int s = 0; s < sweeps; ++s)
    for (int colour = 0; colour < 2; ++colour)
      DD_TIMED("k_sap_colour", st, bytes, flops,
               (k_sap_colour<R, S, Tv, WPE><<<nb, threads, 0, st>>>(g, (const S*)ops.links, (const S*)ops.clover,
                                                               (const S*)ops.cinv, nrhs, colour, mr, (const Tv*)b,
                                                               (Tv*)x)));
}

}  // namespace

void launch_sap(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, int sweeps, int mr_iters, const void* b,
                void* x, int wpe, int dom_rhs, int persist, hipStream_t st) {
  if (dom_rhs > 0 && sap_dom_supported(g, dt)) {   // domain-resident form (sap_dom.hip)
    launch_sap_dom(g, dt, ops, nrhs, sweeps, mr_iters, b, x, dom_rhs, persist != 0, st);
    return;
  }
#define DD_SAP_WPE(R, S, Tv)                                                   \
  switch (wpe) {                                                               \
    case 3: run<R, S, Tv, 3>(g, ops, nrhs, sweeps, mr_iters, b, x, st); break; \
    default: run<R, S, Tv, 2>(g, ops, nrhs, sweeps, mr_iters, b, x, st); break; \
  }
  switch (dt) {
    case DD_F64: run<double, double2, double2, 1>(g, ops, nrhs, sweeps, mr_iters, b, x, st); break;
    case DD_F32: DD_SAP_WPE(float, float2, float2) break;
    case DD_F16: DD_SAP_WPE(float, __half2, float2) break;
    case DD_BF16: DD_SAP_WPE(float, bf16x2, float2) break;
  }
#undef DD_SAP_WPE
}

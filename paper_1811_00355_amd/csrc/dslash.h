// Device building blocks of the Wilson-clover operator (Sec. 3: hopping term
// and clover term), shared by the operator apply, the SAP smoother and the
// coarse-operator construction.
//
// Chiral representation: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] on (upper,
// lower) spin pairs, A_x = -i sigma_1, A_y = -i sigma_2, A_z = -i sigma_3,
// A_t = 1.  A hop with (1 + s gamma_mu) (s = -1 forward, +1 backward) acts on
// the half spinor h = psi_up + s A_mu psi_dn; the lower pair of the result is
// s A_mu^dag h.  So every hop multiplies only two colour vectors by a link.
#pragma once
#include "dd_internal.h"

// o = A_mu d   (d, o: two colour vectors each)
template <int MU, typename R>
__device__ __forceinline__ void A_mul(const cx<R>* d0, const cx<R>* d1, cx<R>* o0, cx<R>* o1) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (MU == 0) { o0[a] = times_mi(d1[a]); o1[a] = times_mi(d0[a]); }
    if (MU == 1) { o0[a] = -d1[a]; o1[a] = d0[a]; }
    if (MU == 2) { o0[a] = times_mi(d0[a]); o1[a] = times_i(d1[a]); }
    if (MU == 3) { o0[a] = d0[a]; o1[a] = d1[a]; }
  }
}
// o = A_mu^dag h
template <int MU, typename R>
__device__ __forceinline__ void Adag_mul(const cx<R>* h0, const cx<R>* h1, cx<R>* o0, cx<R>* o1) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (MU == 0) { o0[a] = times_i(h1[a]); o1[a] = times_i(h0[a]); }
    if (MU == 1) { o0[a] = h1[a]; o1[a] = -h0[a]; }
    if (MU == 2) { o0[a] = times_i(h0[a]); o1[a] = times_mi(h1[a]); }
    if (MU == 3) { o0[a] = h0[a]; o1[a] = h1[a]; }
  }
}

// half spinor h = psi_up + s A_mu psi_dn  (h: 6 complex, spin-major)
template <int MU, int SGN, typename R>
__device__ __forceinline__ void project(const cx<R>* psi, cx<R>* h) {
  cx<R> t0[3], t1[3];
  A_mul<MU, R>(psi + 6, psi + 9, t0, t1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h[a] = (SGN > 0) ? psi[a] + t0[a] : psi[a] - t0[a];
    h[3 + a] = (SGN > 0) ? psi[3 + a] + t1[a] : psi[3 + a] - t1[a];
  }
}

// acc += c * (h, s A_mu^dag h)
template <int MU, int SGN, typename R>
__device__ __forceinline__ void reconstruct_acc(const cx<R>* h, R c, cx<R>* acc) {
  cx<R> t0[3], t1[3];
  Adag_mul<MU, R>(h, h + 3, t0, t1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] = acc[a] + c * h[a];
    acc[3 + a] = acc[3 + a] + c * h[3 + a];
    R cs = (SGN > 0) ? c : -c;
    acc[6 + a] = acc[6 + a] + cs * t0[a];
    acc[9 + a] = acc[9 + a] + cs * t1[a];
  }
}

template <typename R, typename S>
__device__ __forceinline__ void load_link(const S* L, long long V, int mu, long long I, cx<R>* u) {
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = ld<R, S>(L + (long long)(mu * 9 + k) * V + I);
}

// acc += a * b and acc += conj(a) * b as four chained fused multiply-adds (one
// rounding each, 4 VALU operations instead of 6 for sum-then-accumulate); used
// where the hop and clover arithmetic is the bottleneck.
template <typename R>
__device__ __forceinline__ void cfma4(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
template <typename R>
__device__ __forceinline__ void cfma4_conj(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}

// o = U h on both spin components of a half spinor
template <typename R>
__device__ __forceinline__ void su3_mul_half(const cx<R>* u, const cx<R>* h, cx<R>* o) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> acc = u[3 * a] * h[3 * s];
      cfma4(acc, u[3 * a + 1], h[3 * s + 1]);
      cfma4(acc, u[3 * a + 2], h[3 * s + 2]);
      o[3 * s + a] = acc;
    }
}
// o = U^dag h
template <typename R>
__device__ __forceinline__ void su3_dag_mul_half(const cx<R>* u, const cx<R>* h, cx<R>* o) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> acc = cmul_conj(u[a], h[3 * s]);
      cfma4_conj(acc, u[3 + a], h[3 * s + 1]);
      cfma4_conj(acc, u[6 + a], h[3 * s + 2]);
      o[3 * s + a] = acc;
    }
}

// out (=|+=) C psi for a packed clover-like field (two Hermitian 6x6 blocks)
template <typename R, typename S, bool ACC>
__device__ __forceinline__ void clover_mul(const S* C, long long V, long long I, const cx<R>* in, cx<R>* out) {
  // one chirality block at a time (36 reals of operand live, not 72)
#pragma unroll 1
  for (int c = 0; c < 2; ++c) {
    const S* B = C + (long long)(18 * c) * V + I;
    cx<R> v[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) v[r] = c ? in[6 + r] : in[r];
    cx<R> o[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cx<R> d = ld<R, S>(B + k * V);
      o[2 * k] = d.re * v[2 * k];
      o[2 * k + 1] = d.im * v[2 * k + 1];
    }
    int k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = r + 1; q < 6; ++q) {
        cx<R> u = ld<R, S>(B + (long long)(k++) * V);
        cfma4(o[r], u, v[q]);
        cfma4_conj(o[q], u, v[r]);
      }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (c) out[6 + r] = ACC ? out[6 + r] + o[r] : o[r];
      else out[r] = ACC ? out[r] + o[r] : o[r];
    }
  }
}

template <typename R, typename Tv>
__device__ __forceinline__ void load_spinor(const Tv* p, long long V, long long I, cx<R>* psi) {
#pragma unroll
  for (int c = 0; c < 12; ++c) psi[c] = ld<R, Tv>(p + (long long)c * V + I);
}
template <typename R, typename Tv>
__device__ __forceinline__ void store_spinor(Tv* p, long long V, long long I, const cx<R>* psi) {
#pragma unroll
  for (int c = 0; c < 12; ++c) st<Tv, R>(p + (long long)c * V + I, psi[c]);
}

// Runtime-direction form of the same actions.  A_mu d = (c0 d_p0, c1 d_p1) and
// A_mu^dag h = (k0 h_q0, k1 h_q1) with unit complex coefficients; one loop body
// serves all directions, which keeps the live register set to one hop.
struct HopCoef {
  int p0, q0;              // permutation: component index feeding output 0 (1 - it feeds output 1)
  float c0r, c0i, c1r, c1i;   // A_mu coefficients
  float k0r, k0i, k1r, k1i;   // A_mu^dag coefficients
};
__device__ __forceinline__ HopCoef hop_coef(int mu) {
  switch (mu) {
    case 0: return {1, 1, 0.f, -1.f, 0.f, -1.f, 0.f, 1.f, 0.f, 1.f};
    case 1: return {1, 1, -1.f, 0.f, 1.f, 0.f, 1.f, 0.f, -1.f, 0.f};
    case 2: return {0, 0, 0.f, -1.f, 0.f, 1.f, 0.f, 1.f, 0.f, -1.f};
    default: return {0, 0, 1.f, 0.f, 1.f, 0.f, 1.f, 0.f, 1.f, 0.f};
  }
}

template <typename R>
__device__ __forceinline__ cx<R> unit_mul(R cr, R ci, cx<R> a) {
  return {cr * a.re - ci * a.im, cr * a.im + ci * a.re};
}

// acc += scale * phase * (-1/2) (1 + sgn gamma_mu) U psi_nb, with U = U_mu(x)
// (forward, sgn = -1) or U_mu(x - mu)^dag (backward, sgn = +1) already loaded
template <typename R>
__device__ __forceinline__ void hop_rt(const HopCoef& hc, int sgn, bool dag, const cx<R>* u, const cx<R>* psi, R coef,
                                       cx<R>* acc) {
  cx<R> h[6], uh[6];
  // h = psi_up + sgn * A_mu psi_dn   (selects, not indexing, keep everything in registers)
  const R s = (R)sgn;
  const bool swp = hc.p0 != 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> d0 = swp ? psi[9 + a] : psi[6 + a];
    cx<R> d1 = swp ? psi[6 + a] : psi[9 + a];
    h[a] = psi[a] + s * unit_mul<R>((R)hc.c0r, (R)hc.c0i, d0);
    h[3 + a] = psi[3 + a] + s * unit_mul<R>((R)hc.c1r, (R)hc.c1i, d1);
  }
  if (dag) su3_dag_mul_half<R>(u, h, uh);
  else su3_mul_half<R>(u, h, uh);
  // acc += coef * (uh, sgn A_mu^dag uh)
  const R cs = s * coef;
  const bool swq = hc.q0 != 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> e0 = swq ? uh[3 + a] : uh[a];
    cx<R> e1 = swq ? uh[a] : uh[3 + a];
    acc[a] = acc[a] + coef * uh[a];
    acc[3 + a] = acc[3 + a] + coef * uh[3 + a];
    acc[6 + a] = acc[6 + a] + cs * unit_mul<R>((R)hc.k0r, (R)hc.k0i, e0);
    acc[9 + a] = acc[9 + a] + cs * unit_mul<R>((R)hc.k1r, (R)hc.k1i, e1);
  }
}

// One hop with compile-time direction and sign: project to the half spinor,
// multiply by U (forward) or U^dag (backward), reconstruct into acc with coef.
template <int MU, int SGN, bool DAG, typename R>
__device__ __forceinline__ void hop_t(const cx<R>* u, const cx<R>* psi, R coef, cx<R>* acc) {
  cx<R> h[6], uh[6];
  project<MU, SGN, R>(psi, h);
  if (DAG) su3_dag_mul_half<R>(u, h, uh);
  else su3_mul_half<R>(u, h, uh);
  reconstruct_acc<MU, SGN, R>(uh, coef, acc);
}

// acc += scale * (hopping term at site s).  The neighbour spinor is fetched by
// `fetch(J, inside, psi)`; with `dirichlet`, hops to sites outside the block
// are dropped.  The loop over the 8 (direction, sign) pairs stays rolled so
// that only one hop is live in registers; a uniform switch selects the
// compile-time form of each hop, whose gamma-matrix factors are then plain
// swaps and sign flips.
template <typename R, typename S, typename Fetch>
__device__ __forceinline__ void hop_all(const GeomDev& g, const S* links, const SiteLoc& s, long long I, bool dirichlet,
                                        Fetch fetch, cx<R>* acc, R scale = (R)1) {
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const int mu = k >> 1;
    const int sign = (k & 1) ? -1 : +1;
    bool wrap, inside;
    long long J = neighbor(g, s, mu, sign, wrap, inside);
    if (dirichlet && !inside) continue;
    cx<R> psi[12], u[9];
    fetch(J, inside, psi);
    load_link<R, S>(links, g.V, mu, sign > 0 ? I : J, u);
    const R coef = scale * (R)(wrap ? -0.5 * g.bc_t : -0.5);
    // forward (1 - gamma_mu) U_mu(x) psi(x + mu); backward (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
    switch (k) {
      case 0: hop_t<0, -1, false, R>(u, psi, coef, acc); break;
      case 1: hop_t<0, +1, true, R>(u, psi, coef, acc); break;
      case 2: hop_t<1, -1, false, R>(u, psi, coef, acc); break;
      case 3: hop_t<1, +1, true, R>(u, psi, coef, acc); break;
      case 4: hop_t<2, -1, false, R>(u, psi, coef, acc); break;
      case 5: hop_t<2, +1, true, R>(u, psi, coef, acc); break;
      case 6: hop_t<3, -1, false, R>(u, psi, coef, acc); break;
      default: hop_t<3, +1, true, R>(u, psi, coef, acc); break;
    }
  }
}

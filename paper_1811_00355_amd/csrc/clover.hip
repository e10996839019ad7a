// Field preparation: the clover term A(x) from the plaquette leaves and its
// inverse, both stored as two packed Hermitian 6x6 chirality blocks (Sec. 3:
// 6 real diagonal entries plus 15 complex upper-triangle entries per block;
// the full inverse is stored instead of an LU factorisation).  FP64.
#include "dd_internal.h"

namespace {

struct M3 {
  cx<double> a[3][3];
};

__device__ __forceinline__ M3 mul(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cx<double> s = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < 3; ++j) cfma(s, x.a[i][j], y.a[j][k]);
      r.a[i][k] = s;
    }
  return r;
}
__device__ __forceinline__ M3 dag(const M3& x) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) r.a[i][k] = conj(x.a[k][i]);
  return r;
}

__device__ __forceinline__ SiteLoc step(const GeomDev& g, SiteLoc s, int mu, int sign) {
  int v = s.l[mu] + sign;
  if (v < 0 || v >= g.b[mu]) {
    int e = g.blk_nbr[(sign > 0 ? mu : 4 + mu) * g.Vc + s.slot];
    s.slot = e & DD_SLOT_MASK;
    v = (sign > 0) ? 0 : g.b[mu] - 1;
  }
  s.l[mu] = v;
  return s;
}

__device__ __forceinline__ M3 link(const GeomDev& g, const double2* L, const SiteLoc& s, int mu) {
  long long I = ((long long)s.slot << g.lBv) + encode_local(g, s.l);
  M3 u;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 v = L[(long long)(mu * 9 + k) * g.V + I];
    u.a[k / 3][k % 3] = {v.x, v.y};
  }
  return u;
}

// sum of the four leaves of the mu-nu plane at x (same orientation; raw links,
// so the t boundary factor cancels in every closed path)
__device__ M3 leaves(const GeomDev& g, const double2* L, const SiteLoc& x, int mu, int nu) {
  SiteLoc xpm = step(g, x, mu, +1), xpn = step(g, x, nu, +1);
  SiteLoc xmm = step(g, x, mu, -1), xmn = step(g, x, nu, -1);
  SiteLoc xmm_pn = step(g, xmm, nu, +1), xmm_mn = step(g, xmm, nu, -1), xmn_pm = step(g, xmn, mu, +1);
  M3 Umu = link(g, L, x, mu), Unu = link(g, L, x, nu);
  M3 q = mul(mul(Umu, link(g, L, xpm, nu)), mul(dag(link(g, L, xpn, mu)), dag(Unu)));
  M3 t = mul(mul(Unu, dag(link(g, L, xmm_pn, mu))), mul(dag(link(g, L, xmm, nu)), link(g, L, xmm, mu)));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) q.a[i][k] = q.a[i][k] + t.a[i][k];
  t = mul(mul(dag(link(g, L, xmm, mu)), dag(link(g, L, xmm_mn, nu))), mul(link(g, L, xmm_mn, mu), link(g, L, xmn, nu)));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) q.a[i][k] = q.a[i][k] + t.a[i][k];
  t = mul(mul(dag(link(g, L, xmn, nu)), link(g, L, xmn, mu)), mul(link(g, L, xmn_pm, nu), dag(Umu)));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) q.a[i][k] = q.a[i][k] + t.a[i][k];
  return q;
}

// the 2x2 spin blocks of the chiral gamma matrices: gamma_mu = [[0, A_mu], [A_mu^dag, 0]]
__device__ __forceinline__ cx<double> Amat(int mu, int r, int c) {
  switch (mu) {
    case 0: return (r != c) ? cx<double>{0.0, -1.0} : cx<double>{0.0, 0.0};
    case 1: return (r == 0 && c == 1) ? cx<double>{-1.0, 0.0}
                 : (r == 1 && c == 0) ? cx<double>{1.0, 0.0} : cx<double>{0.0, 0.0};
    case 2: return (r != c) ? cx<double>{0.0, 0.0} : (r == 0 ? cx<double>{0.0, -1.0} : cx<double>{0.0, 1.0});
    default: return (r == c) ? cx<double>{1.0, 0.0} : cx<double>{0.0, 0.0};
  }
}

// spin block of gamma_mu gamma_nu on chirality c: c = 0 -> A_mu A_nu^dag, c = 1 -> A_mu^dag A_nu
__device__ __forceinline__ cx<double> gg(int c, int mu, int nu, int r, int s) {
  cx<double> acc = {0.0, 0.0};
  for (int k = 0; k < 2; ++k) {
    if (c == 0) acc = acc + Amat(mu, r, k) * conj(Amat(nu, s, k));
    else acc = acc + conj(Amat(mu, k, r)) * Amat(nu, k, s);
  }
  return acc;
}

__device__ void pack6(const cx<double> B[6][6], double2* out, long long stride) {
  out[0 * stride] = make_double2(B[0][0].re, B[1][1].re);
  out[1 * stride] = make_double2(B[2][2].re, B[3][3].re);
  out[2 * stride] = make_double2(B[4][4].re, B[5][5].re);
  int k = 3;
  for (int r = 0; r < 6; ++r)
    for (int c = r + 1; c < 6; ++c) out[(k++) * stride] = make_double2(B[r][c].re, B[r][c].im);
}

// Gauss-Jordan inverse with partial pivoting (FP64)
__device__ void invert6(const cx<double> A[6][6], cx<double> X[6][6]) {
  cx<double> M[6][12];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 12; ++c)
      M[r][c] = (c < 6) ? A[r][c] : ((c - 6 == r) ? cx<double>{1.0, 0.0} : cx<double>{0.0, 0.0});
  for (int k = 0; k < 6; ++k) {
    int piv = k;
    double best = M[k][k].re * M[k][k].re + M[k][k].im * M[k][k].im;
    for (int r = k + 1; r < 6; ++r) {
      double v = M[r][k].re * M[r][k].re + M[r][k].im * M[r][k].im;
      if (v > best) { best = v; piv = r; }
    }
    if (piv != k)
      for (int c = 0; c < 12; ++c) {
        cx<double> t = M[k][c];
        M[k][c] = M[piv][c];
        M[piv][c] = t;
      }
    cx<double> p = M[k][k];
    double d = p.re * p.re + p.im * p.im;
    cx<double> pinv = {p.re / d, -p.im / d};
    for (int c = 0; c < 12; ++c) M[k][c] = M[k][c] * pinv;
    for (int r = 0; r < 6; ++r) {
      if (r == k) continue;
      cx<double> f = M[r][k];
      for (int c = 0; c < 12; ++c) M[r][c] = M[r][c] - f * M[k][c];
    }
  }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) X[r][c] = M[r][c + 6];
}

__global__ void k_clover(GeomDev g, const double2* __restrict__ L, double m0, double csw,
                         double2* __restrict__ clov, double2* __restrict__ cinv) {
  long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= g.V) return;
  SiteLoc x = decode_site(g, I);
  cx<double> B[2][6][6];
  for (int c = 0; c < 2; ++c)
    for (int r = 0; r < 6; ++r)
      for (int s = 0; s < 6; ++s) B[c][r][s] = (r == s) ? cx<double>{4.0 + m0, 0.0} : cx<double>{0.0, 0.0};
  if (csw != 0.0) {
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        M3 Q = leaves(g, L, x, mu, nu);
        // F = (Q_mu,nu - Q_nu,mu)/8 with Q_nu,mu = Q_mu,nu^dagger
        M3 F;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) F.a[a][b] = 0.125 * (Q.a[a][b] - conj(Q.a[b][a]));
        // A -= (c_sw / 2) (gamma_mu gamma_nu) (x) F_mu,nu  on each chirality block
        for (int c = 0; c < 2; ++c)
          for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) {
              cx<double> s = (0.5 * csw) * gg(c, mu, nu, al, be);
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) B[c][3 * al + a][3 * be + b] = B[c][3 * al + a][3 * be + b] - s * F.a[a][b];
            }
      }
  }
  for (int c = 0; c < 2; ++c) {
    pack6(B[c], clov + (long long)(18 * c) * g.V + I, g.V);
    cx<double> X[6][6];
    invert6(B[c], X);
    pack6(X, cinv + (long long)(18 * c) * g.V + I, g.V);
  }
}

}  // namespace

void launch_clover_build(const GeomDev& g, const double2* links64, double m0, double csw, double2* clover64,
                         double2* cinv64, hipStream_t st) {
  k_clover<<<(unsigned)((g.V + 127) / 128), 128, 0, st>>>(g, links64, m0, csw, clover64, cinv64);
}

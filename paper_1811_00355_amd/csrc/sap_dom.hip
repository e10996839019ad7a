// SAP smoother (Sec. 2), domain-resident form for 4^4 domains with FP16 or BF16
// operands: one workgroup per domain of the launched colour.  The domain's
// links and odd-site clover inverse (and, in the four-RHS form, its clover term)
// are staged in LDS once and serve every right-hand side, which the workgroup
// takes G at a time: thread (q, j) owns the even site j and the odd site j of
// right-hand side q of the group.  Two forms (same arithmetic):
//   G = 4: links, clover and inverse in LDS (141 KB): one workgroup (8 waves) per CU;
//   G = 2: links and inverse in LDS (80 KB), the clover read from memory (L2):
//          two domains' workgroups share a CU, so one's memory waits overlap
//          the other's arithmetic.
// The arithmetic is that of the per-RHS kernel in sap.hip:
//   r_B   = b - D x on the domain (halo of x from the other colour's domains)
//   rhs_e = r_e - H_eo A_oo^-1 r_o            (H: hops inside the domain)
//   MR on S = A_ee - H_eo A_oo^-1 H_oe from e_e = 0, k steps
//   e_o   = A_oo^-1 (r_o - H_oe e_e);  x_B += e
// Hops inside the domain read their link and neighbour from LDS at a per-thread
// neighbour table (eight 8-bit half-domain indices, 0xff outside) computed once;
// only the residual's hops across the domain faces read global memory.
#include <hip/hip_cooperative_groups.h>

#include "dslash.h"
#include "ktimer.h"

namespace {

constexpr int kE = 4;              // domain edge
constexpr int kBv = 256, kBvh = 128;

// local coordinates of the site with parity p and half-domain index j
__device__ __forceinline__ void dom_coords(int p, int j, int l[4]) {
  const int lex2 = j << 1;
  l[1] = (lex2 >> 2) & 3;
  l[2] = (lex2 >> 4) & 3;
  l[3] = lex2 >> 6;
  l[0] = (lex2 & 3) + ((p + l[1] + l[2] + l[3]) & 1);
}

// half-domain index of the neighbour in each of the 8 hop directions
// (k = 2 mu for +mu, 2 mu + 1 for -mu), 0xff when it lies outside the domain;
// bytes 0..3 in lo, 4..7 in hi
__device__ __forceinline__ void dom_neighbours(int p, int j, unsigned& lo, unsigned& hi) {
  int l[4];
  dom_coords(p, j, l);
  lo = hi = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int mu = k >> 1, sg = (k & 1) ? -1 : 1;
    int m[4] = {l[0], l[1], l[2], l[3]};
    m[mu] += sg;
    const unsigned b = (m[mu] < 0 || m[mu] >= kE)
                           ? 0xffu
                           : (unsigned)((m[0] + kE * (m[1] + kE * (m[2] + kE * m[3]))) >> 1);
    if (k < 4) lo |= b << (8 * k);
    else hi |= b << (8 * (k - 4));
  }
}

__device__ __forceinline__ unsigned nb_byte(unsigned lo, unsigned hi, int k) {
  return ((k < 4 ? lo : hi) >> (8 * (k & 3))) & 0xffu;
}

// out = C in for a packed Hermitian pair of 6x6 blocks held in LDS as rows of
// STRIDE pairs (row r of this site at C[r * STRIDE]); the order of operations
// is that of clover_mul
template <typename S, int STRIDE>
__device__ __forceinline__ void clover_lds(const S* C, const cx<float>* in, cx<float>* out) {
#pragma unroll 1
  for (int c = 0; c < 2; ++c) {
    const S* B = C + 18 * c * STRIDE;
    cx<float> v[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) v[r] = c ? in[6 + r] : in[r];
    cx<float> o[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<float> d = ld<float, S>(B + k * STRIDE);
      o[2 * k] = d.re * v[2 * k];
      o[2 * k + 1] = d.im * v[2 * k + 1];
    }
    int k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = r + 1; q < 6; ++q) {
        const cx<float> u = ld<float, S>(B + (k++) * STRIDE);
        cfma4(o[r], u, v[q]);
        cfma4_conj(o[q], u, v[r]);
      }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (c) out[6 + r] = o[r];
      else out[r] = o[r];
    }
  }
}

template <int K>
__device__ __forceinline__ void hop_k(const cx<float>* u, const cx<float>* psi, float coef, cx<float>* acc) {
  // forward (1 - gamma_mu) U_mu(x) psi(x + mu); backward (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
  hop_t<K / 2, (K & 1) ? +1 : -1, (K & 1) != 0, float>(u, psi, coef, acc);
}

__device__ __forceinline__ void hop_case(int k, const cx<float>* u, const cx<float>* psi, float coef,
                                         cx<float>* acc) {
  switch (k) {
    case 0: hop_k<0>(u, psi, coef, acc); break;
    case 1: hop_k<1>(u, psi, coef, acc); break;
    case 2: hop_k<2>(u, psi, coef, acc); break;
    case 3: hop_k<3>(u, psi, coef, acc); break;
    case 4: hop_k<4>(u, psi, coef, acc); break;
    case 5: hop_k<5>(u, psi, coef, acc); break;
    case 6: hop_k<6>(u, psi, coef, acc); break;
    default: hop_k<7>(u, psi, coef, acc); break;
  }
}

__device__ __forceinline__ cx<float> unpack(__half2 v) {
  const float2 f = __half22float2(v);
  return {f.x, f.y};
}
__device__ __forceinline__ cx<float> unpack(bf16x2 v) {
  return {__uint_as_float(v.u << 16), __uint_as_float(v.u & 0xffff0000u)};
}

// acc += scale * (hops of site (P, j) to neighbours inside the domain), the
// neighbours' spinors read from X[c * kBvh + half index] (the other parity).
// Branch-free and unrolled: a lane whose neighbour is outside reads site 0 and
// adds it with coefficient 0 (the wave executes that hop for its other lanes
// anyway), so the compiler can issue the reads of later hops early.
template <typename S, int P>
__device__ __forceinline__ void hops_inside(const S* Ls, int j, unsigned lo, unsigned hi, const cx<float>* X,
                                            float scale, cx<float>* acc) {
  const float coef = -0.5f * scale;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const unsigned nbr = nb_byte(lo, hi, k);
    const bool in = nbr != 0xffu;
    const int nb = in ? (int)nbr : 0;
    cx<float> psi[12], u[9];
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = X[c * kBvh + nb];
    // forward: this site's link; backward: the neighbour's link in the same direction
    const int li = (k & 1) ? (1 - P) * kBvh + nb : P * kBvh + j;
    const S* Lk = Ls + (k >> 1) * 9 * kBv + li;
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = unpack(Lk[e * kBv]);
    hop_case(k, u, psi, in ? coef : 0.f, acc);
  }
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// acc += scale * (all eight hops of the site (P, j) of the domain at `slot`):
// neighbours inside the domain from X (the other parity) with the links in LDS,
// neighbours across the faces from the global vector x and, for backward hops,
// the global links.  Kept rolled (one hop's operands live at a time): the
// register budget of the kernel leaves no room to keep the face reads of
// several hops in flight, and the forms that tried were slower.
template <typename S, int P>
__device__ __forceinline__ void hops_residual(const GeomDev& g, const S* __restrict__ links_g, const S* Ls, int slot,
                                              int j, unsigned lo, unsigned hi, const cx<float>* X,
                                              const float2* __restrict__ x, float scale, cx<float>* acc) {
  const long long V = g.V;
  SiteLoc s;
  s.slot = slot;
  dom_coords(P, j, s.l);
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const unsigned nb = nb_byte(lo, hi, k);
    const int mu = k >> 1;
    cx<float> psi[12], u[9];
    float coef = -0.5f * scale;
    if (nb != 0xffu) {
#pragma unroll
      for (int c = 0; c < 12; ++c) psi[c] = X[c * kBvh + nb];
      const int li = (k & 1) ? (1 - P) * kBvh + (int)nb : P * kBvh + j;
      const S* Lk = Ls + mu * 9 * kBv + li;
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = ld<float, S>(Lk + e * kBv);
    } else {
      bool wrap, inside;
      const long long J = neighbor(g, s, mu, (k & 1) ? -1 : 1, wrap, inside);
      load_spinor<float, float2>(x, V, J, psi);
      if (k & 1) {
        load_link<float, S>(links_g, V, mu, J, u);
      } else {
        const S* Lk = Ls + mu * 9 * kBv + P * kBvh + j;
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = ld<float, S>(Lk + e * kBv);
      }
      if (wrap) coef *= (float)g.bc_t;
    }
    hop_case(k, u, psi, coef, acc);
  }
}

// sum over the two waves of right-hand side q (lanes of both waves get the sum)
__device__ __forceinline__ void pair_sum3(float& a, float& b, float& c, float (*red)[2][4], int q, int w,
                                          int lane) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
    c += __shfl_xor(c, off, 64);
  }
  if (lane == 0) {
    red[q][w][0] = a;
    red[q][w][1] = b;
    red[q][w][2] = c;
  }
  __syncthreads();
  a = red[q][0][0] + red[q][1][0];
  b = red[q][0][1] + red[q][1][1];
  c = red[q][0][2] + red[q][1][2];
}

// PERSIST: one cooperative launch runs every sweep and both colours; its
// workgroups (as many as the CUs hold at once) take the domains of a colour in
// turn, contiguous ranges per XCD, and meet at a grid barrier after each
// colour.  Each domain is computed exactly as in the launch-per-colour form
// (domains of one colour are independent), so the results are the same bits.
template <typename S, int G, bool CG, bool PERSIST>
__global__ void __launch_bounds__(kBvh * G) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_sap_dom(GeomDev g, const S* __restrict__ links, const S* __restrict__ clov, const S* __restrict__ cinv, int nrhs,
          int colour0, int sweeps, int mr_iters, const float2* __restrict__ bvec, float2* __restrict__ xvec) {
  __shared__ S sL[36 * kBv];        // links [mu][9][site]
  __shared__ S sC[CG ? 1 : 36 * kBv];   // clover [36][site] (CG: read from memory instead)
  __shared__ S sI[36 * kBvh];       // inverse of the odd sites [36][half index]
  __shared__ cx<float> sX[G][12 * kBvh];   // per right-hand side: one half-domain spinor field
  __shared__ float red[G][2][4];

  const long long V = g.V;
  // q (the right-hand side slot) is uniform over a wave: keep it, and the
  // buffer descriptors derived from it, in scalar registers
  const int t = threadIdx.x, q = __builtin_amdgcn_readfirstlane(t / kBvh), j = t % kBvh, w = (t / 64) & 1,
            lane = t & 63;

  auto domain = [&](int tile, int colour) {
  const int slot = colour * g.Vch + tile;
  const long long base = (long long)slot * kBv;

  // stage the domain's operator: 36 rows of 256 pairs (links; clover unless CG),
  // 36 rows of 128 (odd inverse), in 16-byte pieces, all loads issued before the
  // LDS writes
  {
    constexpr int kRowQ = kBv / 4, kRowQh = kBvh / 4;             // 16-byte pieces per row
    constexpr int kNL = 36 * kRowQ, kNI = 36 * kRowQh;            // pieces per field
    constexpr int kNF = CG ? 1 : 2;                               // full-domain fields staged
    constexpr int kTot = kNF * kNL + kNI;
    constexpr int kPer = (kTot + kBvh * G - 1) / (kBvh * G);
    u32x4 v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = t + i * kBvh * G;
      const int f = e < kNL ? 0 : (e < kNF * kNL ? 1 : 2), r = e < kNF * kNL ? e - f * kNL : e - kNF * kNL;
      const int row = f < 2 ? r / kRowQ : r / kRowQh, q4 = f < 2 ? r % kRowQ : r % kRowQh;
      const S* src = f == 0 ? links : f == 1 ? clov : cinv;
      const long long gi = (long long)row * V + base + (f == 2 ? kBvh : 0) + 4 * q4;
      if (e < kTot) v[i] = *reinterpret_cast<const u32x4*>(src + gi);
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = t + i * kBvh * G;
      const int f = e < kNL ? 0 : (e < kNF * kNL ? 1 : 2), r = e < kNF * kNL ? e - f * kNL : e - kNF * kNL;
      S* dst = f == 0 ? sL : f == 1 ? sC : sI;
      if (e < kTot) *reinterpret_cast<u32x4*>(dst + 4 * r) = v[i];
    }
  }
  unsigned elo, ehi, olo, ohi;
  dom_neighbours(0, j, elo, ehi);
  dom_neighbours(1, j, olo, ohi);
  const long long Ie = base + j, Io = base + kBvh + j;
  cx<float>* X = sX[q];

#pragma unroll 1
  for (int r0 = 0; r0 < nrhs; r0 += G) {
    const int r = r0 + q;
    const bool act = r < nrhs;   // uniform over the two waves of q
    const float2* b = bvec + (long long)(act ? r : 0) * 12 * V;
    float2* x = xvec + (long long)(act ? r : 0) * 12 * V;
    cx<float> ro[12], rho[12], e[12], tt[12];
    __syncthreads();   // the operator is staged; the previous group's reads of X are done
    // x_e to X for the odd sites' hops
    if (act) {
      load_spinor<float, float2>(x, V, Ie, tt);
#pragma unroll
      for (int c = 0; c < 12; ++c) X[c * kBvh + j] = tt[c];
    }
    __syncthreads();
    if (act) {
      // r_o = b_o - A_oo x_o - H x  (x_o kept in rho for the even sites' hops)
      load_spinor<float, float2>(x, V, Io, rho);
      if constexpr (CG) clover_mul<float, S, false>(clov, V, Io, rho, tt);
      else clover_lds<S, kBv>(sC + kBvh + j, rho, tt);
      load_spinor<float, float2>(b, V, Io, ro);
#pragma unroll
      for (int c = 0; c < 12; ++c) ro[c] = ro[c] - tt[c];
      hops_residual<S, 1>(g, links, sL, slot, j, olo, ohi, X, x, -1.f, ro);
    }
    __syncthreads();
    if (act) {
      // x_o (still in rho) to X for the even sites' hops
#pragma unroll
      for (int c = 0; c < 12; ++c) X[c * kBvh + j] = rho[c];
    }
    __syncthreads();
    if (act) {
      // r_e = b_e - A_ee x_e - H x, then A_oo^-1 r_o for the source projection
      load_spinor<float, float2>(x, V, Ie, e);
      if constexpr (CG) clover_mul<float, S, false>(clov, V, Ie, e, tt);
      else clover_lds<S, kBv>(sC + j, e, tt);
      load_spinor<float, float2>(b, V, Ie, rho);
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = rho[c] - tt[c];
      hops_residual<S, 0>(g, links, sL, slot, j, elo, ehi, X, x, -1.f, rho);
      clover_lds<S, kBvh>(sI + j, ro, tt);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 12; ++c) X[c * kBvh + j] = tt[c];
    }
    __syncthreads();
    if (act) {
      // rhs_e = r_e - H_eo A_oo^-1 r_o; MR from e_e = 0 with rho = rhs_e
      hops_inside<S, 0>(sL, j, elo, ehi, X, -1.f, rho);
#pragma unroll
      for (int c = 0; c < 12; ++c) e[c] = {0.f, 0.f};
    }
#pragma unroll 1
    for (int k = 0; k < mr_iters; ++k) {
      __syncthreads();
      if (act) {
#pragma unroll
        for (int c = 0; c < 12; ++c) X[c * kBvh + j] = rho[c];
      }
      __syncthreads();
      cx<float> u[12];
      if (act) {
        // odd: u = A_oo^-1 H_oe rho
#pragma unroll
        for (int c = 0; c < 12; ++c) tt[c] = {0.f, 0.f};
        hops_inside<S, 1>(sL, j, olo, ohi, X, 1.f, tt);
        clover_lds<S, kBvh>(sI + j, tt, u);
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int c = 0; c < 12; ++c) X[c * kBvh + j] = u[c];
      }
      __syncthreads();
      float pr_re = 0.f, pr_im = 0.f, pp = 0.f;
      if (act) {
        // even: p = A_ee rho - H_eo u   (kept in tt)
        if constexpr (CG) clover_mul<float, S, false>(clov, V, Ie, rho, tt);
        else clover_lds<S, kBv>(sC + j, rho, tt);
        hops_inside<S, 0>(sL, j, elo, ehi, X, -1.f, tt);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const cx<float> z = cmul_conj(tt[c], rho[c]);   // conj(p) rho
          pr_re += z.re;
          pr_im += z.im;
          pp += tt[c].re * tt[c].re + tt[c].im * tt[c].im;
        }
      }
      pair_sum3(pr_re, pr_im, pp, red, q, w, lane);
      if (act) {
        cx<float> alpha = {0.f, 0.f};
        if (pp > 0.f) alpha = {pr_re / pp, pr_im / pp};
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          cfma(e[c], alpha, rho[c]);
          rho[c] = rho[c] - alpha * tt[c];
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 12; ++c) X[c * kBvh + j] = e[c];
    }
    __syncthreads();
    if (act) {
      // x_e += e_e
      load_spinor<float, float2>(x, V, Ie, tt);
#pragma unroll
      for (int c = 0; c < 12; ++c) tt[c] = tt[c] + e[c];
      store_spinor<float, float2>(x, V, Ie, tt);
      // e_o = A_oo^-1 (r_o - H_oe e_e);  x_o += e_o
      hops_inside<S, 1>(sL, j, olo, ohi, X, -1.f, ro);
      clover_lds<S, kBvh>(sI + j, ro, tt);
      load_spinor<float, float2>(x, V, Io, rho);
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = rho[c] + tt[c];
      store_spinor<float, float2>(x, V, Io, rho);
    }
  }
  };

  if constexpr (!PERSIST) {
    // domains of one colour in lexicographic block order, contiguous ranges per XCD
    int tile, unused;
    xcd_range_tile(g.Vch, 1, tile, unused);
    if (tile >= g.Vch) return;   // uniform per workgroup
    domain(tile, colour0);
  } else {
    // gridDim.x is a multiple of 8 and at most Vch; workgroup k of XCD x takes
    // domains k, k + gridDim.x / 8, ... of that XCD's eighth
    const int per_x = g.Vch / 8, nwx = gridDim.x / 8, x8 = blockIdx.x & 7, k0 = blockIdx.x >> 3;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
#pragma unroll 1
    for (int sw = 0; sw < sweeps; ++sw)
#pragma unroll 1
      for (int colour = 0; colour < 2; ++colour) {
#pragma unroll 1
        for (int k = k0; k < per_x; k += nwx) {
          __syncthreads();   // the previous domain's LDS reads are done before the staging overwrites them
          domain(x8 * per_x + k, colour);
        }
        grid.sync();         // the colour's updates of x are visible to the other colour
      }
  }
}

// workgroups of the persistent form: as many as the CUs hold at once (a
// multiple of 8, at most one per domain of a colour); 0 if it cannot be launched
template <typename S, int G, bool CG>
int persist_grid(const GeomDev& g) {
  static thread_local int cached = -1;
  static thread_local long long cached_vch = -1;
  if (cached >= 0 && cached_vch == g.Vch) return cached;
  int dev = 0, ncu = 0, per_cu = 0, coop = 0;
  int n = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sap_dom<S, G, CG, true>, kBvh * G, 0) == hipSuccess) {
    const long long cap = (long long)ncu * per_cu;
    n = (int)((cap < g.Vch ? cap : g.Vch) / 8 * 8);
  }
  (void)hipGetLastError();
  cached = n;
  cached_vch = g.Vch;
  return n;
}

template <typename S, int G, bool CG>
void run_dom(const GeomDev& g, const OpSet& ops, int nrhs, int sweeps, int mr, const void* b, void* x, bool persist,
             hipStream_t st) {
  const double half = 0.5 * (double)g.V;
  const double bytes = half * (90.0 * sizeof(S) + 36.0 * sizeof(float2) * nrhs);
  const double flops = half * nrhs * (mr + 2.5) * 1850.0;
  const S* L = (const S*)ops.links;
  const S* C = (const S*)ops.clover;
  const S* I = (const S*)ops.cinv;
  const float2* bb = (const float2*)b;
  float2* xx = (float2*)x;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(st, &cs);
  const int pg = persist && cs == hipStreamCaptureStatusNone ? persist_grid<S, G, CG>(g) : 0;
  if (pg > 0) {
    GeomDev gg = g;
    int nr = nrhs, c0 = 0, sw = sweeps, mr_ = mr;
    void* args[] = {&gg, &L, &C, &I, &nr, &c0, &sw, &mr_, &bb, &xx};
    DD_TIMED("k_sap_dom_persist", st, bytes * 2 * sweeps, flops * 2 * sweeps,
             (void)hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sap_dom<S, G, CG, true>), dim3(pg),
                                              dim3(kBvh * G), args, 0, st));
    return;
  }
  const unsigned nb = xcd_grid(g.Vch, 1);
  for (int s = 0; s < sweeps; ++s)
    for (int colour = 0; colour < 2; ++colour)
      DD_TIMED("k_sap_dom", st, bytes, flops,
               (k_sap_dom<S, G, CG, false><<<nb, kBvh * G, 0, st>>>(g, L, C, I, nrhs, colour, 1, mr, bb, xx)));
}

}  // namespace

bool sap_dom_supported(const GeomDev& g, dd_dtype dt) {
  return (dt == DD_F16 || dt == DD_BF16) && g.b[0] == kE && g.b[1] == kE && g.b[2] == kE && g.b[3] == kE &&
         g.Vch % 8 == 0;
}

void launch_sap_dom(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, int sweeps, int mr_iters,
                    const void* b, void* x, int rhs_group, bool persist, hipStream_t st) {
  if (rhs_group == 2) {
    if (dt == DD_F16) run_dom<__half2, 2, true>(g, ops, nrhs, sweeps, mr_iters, b, x, persist, st);
    else run_dom<bf16x2, 2, true>(g, ops, nrhs, sweeps, mr_iters, b, x, persist, st);
  } else {
    if (dt == DD_F16) run_dom<__half2, 4, false>(g, ops, nrhs, sweeps, mr_iters, b, x, persist, st);
    else run_dom<bf16x2, 4, false>(g, ops, nrhs, sweeps, mr_iters, b, x, persist, st);
  }
}

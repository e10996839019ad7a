// Wilson-clover operator apply: out = A psi + hopping term (Sec. 3), one
// thread per (site, right-hand side).  Tiles are visited in slab order: the
// workgroups of one tile (all right-hand sides) run on the same XCD back to back,
// so its links and clover come from that XCD's L2 after the first fetch, and
// neighbouring blocks run together on that XCD, so halo spinors and backward
// links are shared through the same L2.  Lattices with 4^4 blocks take the
// block form (k_dirac_blk), whose in-block hops read spinors staged in LDS.
#include "dslash.h"
#include "ktimer.h"

namespace {

template <typename R, typename S, typename Tv, typename To = Tv>
__global__ void __launch_bounds__(256) k_dirac(GeomDev g, const S* __restrict__ links, const S* __restrict__ clov,
                                               int nrhs, const Tv* __restrict__ in, To* __restrict__ out) {
  int tile, r;
  if (g.Bv >= (int)blockDim.x) {   // whole blocks per tile range: slab order (see xcd_slab_tile)
    if (!xcd_slab_tile(g, g.Bv / blockDim.x, nrhs, tile, r)) return;
  } else {
    xcd_tile_rhs(nrhs, tile, r);
  }
  long long I = (long long)tile * blockDim.x + threadIdx.x;
  if (I >= g.V) return;
  const Tv* x = in + (long long)r * 12 * g.V;
  SiteLoc s = decode_site(g, I);
  cx<R> psi[12], acc[12];
  load_spinor<R, Tv>(x, g.V, I, psi);
  clover_mul<R, S, false>(clov, g.V, I, psi, acc);
  auto fetch = [&](long long J, bool, cx<R>* p) { load_spinor<R, Tv>(x, g.V, J, p); };
  hop_all<R, S>(g, links, s, I, false, fetch, acc);
  store_spinor<R, To>(out + (long long)r * 12 * g.V, g.V, I, acc);
}

// With one right-hand side the streams read or written once per launch (the
// clover operand, the output spinor) take non-temporal accesses, so that L2
// keeps what neighbouring sites read again: the links (a site's forward link
// is its backward neighbour's backward link) and the face spinors of
// neighbouring blocks.  With several right-hand sides each RHS's workgroup
// re-reads the clover, and L2 should keep it.
template <typename R, typename S>
__device__ __forceinline__ cx<R> ld_stream(const S* p) {
  return ld<R, S>(p);
}
template <>
__device__ __forceinline__ cx<double> ld_stream<double, double2>(const double2* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ cx<float> ld_stream<float, float2>(const float2* p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return {v.x, v.y};
}
template <typename To, typename R>
__device__ __forceinline__ void st_stream(To* p, cx<R> v) {
  st<To, R>(p, v);
}
template <>
__device__ __forceinline__ void st_stream<double2, double>(double2* p, cx<double> v) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2{v.re, v.im}, reinterpret_cast<v2*>(p));
}
template <>
__device__ __forceinline__ void st_stream<float2, float>(float2* p, cx<float> v) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2{v.re, v.im}, reinterpret_cast<v2*>(p));
}

// C psi for the packed clover (two Hermitian 6x6 blocks), operand read as a stream
template <typename R, typename S>
__device__ __forceinline__ void clover_mul_stream(const S* C, long long V, long long I, const cx<R>* in,
                                                  cx<R>* out) {
#pragma unroll 1
  for (int c = 0; c < 2; ++c) {
    const S* B = C + (long long)(18 * c) * V + I;
    cx<R> v[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) v[r] = c ? in[6 + r] : in[r];
    cx<R> o[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<R> d = ld_stream<R, S>(B + k * V);
      o[2 * k] = d.re * v[2 * k];
      o[2 * k + 1] = d.im * v[2 * k + 1];
    }
    int k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = r + 1; q < 6; ++q) {
        const cx<R> u = ld_stream<R, S>(B + (long long)(k++) * V);
        cfma4(o[r], u, v[q]);
        cfma4_conj(o[q], u, v[r]);
      }
#pragma unroll
    for (int r = 0; r < 6; ++r) {   // constant indices (c is not unrolled): acc stays in registers
      if (c) out[6 + r] = o[r];
      else out[r] = o[r];
    }
  }
}

// The eight hops in the order of hop_all (forward then backward per direction),
// with both links of a direction loaded together: the backward neighbour's
// forward link U_mu(x - mu) lies, for most sites, in the lines the workgroup's
// own forward loads have just fetched, which the L2 does not keep until a
// later backward hop once many blocks stream through it.
template <typename R, typename S, typename Fetch>
__device__ __forceinline__ void hop_pairs(const GeomDev& g, const S* links, const SiteLoc& s, long long I,
                                          Fetch fetch, cx<R>* acc) {
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    bool wf, inf, wb, inb;
    const long long Jf = neighbor(g, s, mu, +1, wf, inf);
    const long long Jb = neighbor(g, s, mu, -1, wb, inb);
    cx<R> uf[9], ub[9], psi[12];
    load_link<R, S>(links, g.V, mu, I, uf);
    load_link<R, S>(links, g.V, mu, Jb, ub);
    fetch(Jf, inf, psi);
    const R cf = (R)1 * (R)(wf ? -0.5 * g.bc_t : -0.5);
    switch (mu) {
      case 0: hop_t<0, -1, false, R>(uf, psi, cf, acc); break;
      case 1: hop_t<1, -1, false, R>(uf, psi, cf, acc); break;
      case 2: hop_t<2, -1, false, R>(uf, psi, cf, acc); break;
      default: hop_t<3, -1, false, R>(uf, psi, cf, acc); break;
    }
    fetch(Jb, inb, psi);
    const R cb = (R)1 * (R)(wb ? -0.5 * g.bc_t : -0.5);
    switch (mu) {
      case 0: hop_t<0, +1, true, R>(ub, psi, cb, acc); break;
      case 1: hop_t<1, +1, true, R>(ub, psi, cb, acc); break;
      case 2: hop_t<2, +1, true, R>(ub, psi, cb, acc); break;
      default: hop_t<3, +1, true, R>(ub, psi, cb, acc); break;
    }
  }
}

// Block form (4^4 blocks: one workgroup of Bv = 256 threads per block and
// right-hand side).  The block's spinors are staged in LDS once; hops to sites
// of the same block read them there, so memory sees one read of every spinor
// plus the hops across the block faces (a quarter of the sites per direction),
// instead of eight gathers per site that the L2 cannot hold between hops.
template <typename R, typename S, typename Tv, typename To = Tv, bool NT = false>
__global__ void __launch_bounds__(256) k_dirac_blk(GeomDev g, const S* __restrict__ links,
                                                   const S* __restrict__ clov, int nrhs, const Tv* __restrict__ in,
                                                   To* __restrict__ out) {
  __shared__ cx<R> sp[12][256];
  int tile, r;
  if (!xcd_slab_tile(g, 1, nrhs, tile, r)) return;   // uniform per workgroup
  const long long base = (long long)tile * 256;
  const long long I = base + threadIdx.x;
  const Tv* x = in + (long long)r * 12 * g.V;
  SiteLoc s = decode_site(g, I);
  cx<R> psi[12], acc[12];
  load_spinor<R, Tv>(x, g.V, I, psi);
#pragma unroll
  for (int c = 0; c < 12; ++c) sp[c][threadIdx.x] = psi[c];
  __syncthreads();
  if constexpr (NT) clover_mul_stream<R, S>(clov, g.V, I, psi, acc);
  else clover_mul<R, S, false>(clov, g.V, I, psi, acc);
  auto fetch = [&](long long J, bool inside, cx<R>* p) {
    if (inside) {
      const int j = (int)(J - base);
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c] = sp[c][j];
    } else {
      load_spinor<R, Tv>(x, g.V, J, p);
    }
  };
  hop_pairs<R, S>(g, links, s, I, fetch, acc);
  To* o = out + (long long)r * 12 * g.V;
  if constexpr (NT) {
#pragma unroll
    for (int c = 0; c < 12; ++c) st_stream<To, R>(o + (long long)c * g.V + I, acc[c]);
  } else {
    store_spinor<R, To>(o, g.V, I, acc);
  }
}

// Half-precision operands, several right-hand sides (4^4 blocks): one workgroup
// per block takes every right-hand side in turn.  A site's 8 links (4 forward,
// the 4 backward U_mu(x - mu)) stay in registers in their storage type (72
// 32-bit registers) and the block's packed clover in LDS, both loaded once, so
// links and clover are read once per launch instead of once per right-hand
// side.  Each right-hand side's block spinors are staged in LDS; hops across the
// block faces read memory.  Same arithmetic, in the same order, as k_dirac_blk.
template <typename S, int STRIDE>
__device__ __forceinline__ void clover_rows(const S* C, const cx<float>* in, cx<float>* out) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const S* B = C + 18 * c * STRIDE;
    cx<float> v[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) v[r] = in[6 * c + r];
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
    for (int r = 0; r < 6; ++r) out[6 * c + r] = o[r];
  }
}

template <typename S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_dirac_hl(
    GeomDev g, const S* __restrict__ links, const S* __restrict__ clov, int nrhs, const float2* __restrict__ in,
    float2* __restrict__ out) {
  __shared__ cx<float> sp[12][256];
  __shared__ S sc[36][256];
  int tile, unused;
  if (!xcd_slab_tile(g, 1, 1, tile, unused)) return;   // uniform per workgroup
  const long long V = g.V, base = (long long)tile * 256, I = base + threadIdx.x;
  const SiteLoc s = decode_site(g, I);
  unsigned J[8];   // packed neighbour indices (V < 2^32)
  unsigned inside = 0, wrap = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    bool w, in_;
    J[k] = (unsigned)neighbor(g, s, k >> 1, (k & 1) ? -1 : +1, w, in_);
    inside |= (unsigned)in_ << k;
    wrap |= (unsigned)w << k;
  }
  S u[8][9];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int e = 0; e < 9; ++e)
      u[k][e] = links[(long long)((k >> 1) * 9 + e) * V + ((k & 1) ? (long long)J[k] : I)];
#pragma unroll
  for (int e = 0; e < 36; ++e) sc[e][threadIdx.x] = clov[(long long)e * V + I];
#pragma unroll 1
  for (int r = 0; r < nrhs; ++r) {
    const float2* x = in + (long long)r * 12 * V;
    cx<float> psi[12], acc[12];
    load_spinor<float, float2>(x, V, I, psi);
    __syncthreads();   // the previous right-hand side's reads of sp are done
#pragma unroll
    for (int c = 0; c < 12; ++c) sp[c][threadIdx.x] = psi[c];
    __syncthreads();
    clover_rows<S, 256>(&sc[0][threadIdx.x], psi, acc);
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      cx<float> nb[12], uk[9];
      if ((inside >> k) & 1) {
        const int jl = (int)(J[k] - (unsigned)base);
#pragma unroll
        for (int c = 0; c < 12; ++c) nb[c] = sp[c][jl];
      } else {
        load_spinor<float, float2>(x, V, (long long)J[k], nb);
      }
      const float coef = -0.5f * (((wrap >> k) & 1) ? (float)g.bc_t : 1.f);
      switch (k) {
#define DD_HOP(K, MU, SG, DG)                                                      \
  case K:                                                                         \
    _Pragma("unroll") for (int e = 0; e < 9; ++e) uk[e] = ld<float, S>(&u[K][e]); \
    hop_t<MU, SG, DG, float>(uk, nb, coef, acc);                                  \
    break;
        DD_HOP(0, 0, -1, false)
        DD_HOP(1, 0, +1, true)
        DD_HOP(2, 1, -1, false)
        DD_HOP(3, 1, +1, true)
        DD_HOP(4, 2, -1, false)
        DD_HOP(5, 2, +1, true)
        DD_HOP(6, 3, -1, false)
        default: DD_HOP(7, 3, +1, true)
#undef DD_HOP
      }
    }
    store_spinor<float, float2>(out + (long long)r * 12 * V, V, I, acc);
  }
}

// useful flops of one site's D apply: eight hops (project, SU(3) times a half
// spinor, reconstruct and accumulate: 1320), the two packed 6x6 clover blocks
// (504) and the final sum (24)
constexpr double kDiracFlopsPerSite = 1320.0 + 504.0 + 24.0;

}  // namespace

// block form of every storage type; NT: streaming clover and output (one right-hand side)
template <bool NT>
static void blk_dispatch(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, const void* in, void* out,
                         hipStream_t st) {
  const unsigned nb = xcd_grid(g.Vc, nrhs);
  switch (dt) {
    case DD_F64:
      k_dirac_blk<double, double2, double2, double2, NT><<<nb, 256, 0, st>>>(
          g, (const double2*)ops.links, (const double2*)ops.clover, nrhs, (const double2*)in, (double2*)out);
      break;
    case DD_F32:
      k_dirac_blk<float, float2, float2, float2, NT><<<nb, 256, 0, st>>>(
          g, (const float2*)ops.links, (const float2*)ops.clover, nrhs, (const float2*)in, (float2*)out);
      break;
    case DD_F16:
      k_dirac_blk<float, __half2, float2, float2, NT><<<nb, 256, 0, st>>>(
          g, (const __half2*)ops.links, (const __half2*)ops.clover, nrhs, (const float2*)in, (float2*)out);
      break;
    case DD_BF16:
      k_dirac_blk<float, bf16x2, float2, float2, NT><<<nb, 256, 0, st>>>(
          g, (const bf16x2*)ops.links, (const bf16x2*)ops.clover, nrhs, (const float2*)in, (float2*)out);
      break;
  }
}

static void dirac_dispatch(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, const void* in, void* out,
                           int threads, hipStream_t st) {
  if (g.Bv == 256 && g.Vc % 16 == 0 && nrhs >= 2 && (dt == DD_F16 || dt == DD_BF16)) {
    // operator in registers across the right-hand sides
    const unsigned nb = xcd_grid(g.Vc, 1);
    if (dt == DD_F16)
      k_dirac_hl<__half2><<<nb, 256, 0, st>>>(g, (const __half2*)ops.links, (const __half2*)ops.clover, nrhs,
                                               (const float2*)in, (float2*)out);
    else
      k_dirac_hl<bf16x2><<<nb, 256, 0, st>>>(g, (const bf16x2*)ops.links, (const bf16x2*)ops.clover, nrhs,
                                              (const float2*)in, (float2*)out);
    return;
  }
  if (g.Bv == 256 && g.Vc % 16 == 0) {   // block form, slab order over the blocks
    if (nrhs == 1)
      blk_dispatch<true>(g, dt, ops, nrhs, in, out, st);
    else
      blk_dispatch<false>(g, dt, ops, nrhs, in, out, st);
    return;
  }
  if (threads != 64 && threads != 128) threads = 256;
  unsigned nb = xcd_grid((unsigned)((g.V + threads - 1) / threads), nrhs);
  switch (dt) {
    case DD_F64:
      k_dirac<double, double2, double2><<<nb, threads, 0, st>>>(g, (const double2*)ops.links, (const double2*)ops.clover,
                                                            nrhs, (const double2*)in, (double2*)out);
      break;
    case DD_F32:
      k_dirac<float, float2, float2><<<nb, threads, 0, st>>>(g, (const float2*)ops.links, (const float2*)ops.clover, nrhs,
                                                         (const float2*)in, (float2*)out);
      break;
    case DD_F16:
      k_dirac<float, __half2, float2><<<nb, threads, 0, st>>>(g, (const __half2*)ops.links, (const __half2*)ops.clover,
                                                          nrhs, (const float2*)in, (float2*)out);
      break;
    case DD_BF16:
      k_dirac<float, bf16x2, float2><<<nb, threads, 0, st>>>(g, (const bf16x2*)ops.links, (const bf16x2*)ops.clover, nrhs,
                                                         (const float2*)in, (float2*)out);
      break;
  }
}

void launch_dirac(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, const void* in, void* out,
                  hipStream_t st, int threads) {
  // algorithmic traffic: spinor in + out per RHS, 4 links + packed clover once per site
  double bytes = (double)g.V * (24.0 * vector_pair_bytes(dt) * nrhs + 72.0 * storage_pair_bytes(dt));
  double flops = (double)g.V * nrhs * kDiracFlopsPerSite;
  DD_TIMED("k_dirac", st, bytes, flops, dirac_dispatch(g, dt, ops, nrhs, in, out, threads, st));
}

void launch_dirac_f32_in(const GeomDev& g, const OpSet& ops64, int nrhs, const float2* in, double2* out,
                         hipStream_t st, int threads) {
  // FP64 operator on an FP32 input (widened exactly on load), FP64 output
  const double bytes = (double)g.V * (12.0 * (sizeof(float2) + sizeof(double2)) * nrhs + 72.0 * sizeof(double2));
  const double flops = (double)g.V * nrhs * kDiracFlopsPerSite;
  const double2* L = (const double2*)ops64.links;
  const double2* C = (const double2*)ops64.clover;
  if (g.Bv == 256 && g.Vc % 16 == 0) {
    if (nrhs == 1)
      DD_TIMED("k_dirac", st, bytes, flops,
               (k_dirac_blk<double, double2, float2, double2, true><<<xcd_grid(g.Vc, nrhs), 256, 0, st>>>(
                   g, L, C, nrhs, in, out)));
    else
      DD_TIMED("k_dirac", st, bytes, flops,
               (k_dirac_blk<double, double2, float2, double2, false><<<xcd_grid(g.Vc, nrhs), 256, 0, st>>>(
                   g, L, C, nrhs, in, out)));
    return;
  }
  if (threads != 64 && threads != 128) threads = 256;
  const unsigned nb = xcd_grid((unsigned)((g.V + threads - 1) / threads), nrhs);
  DD_TIMED("k_dirac", st, bytes, flops,
           (k_dirac<double, double2, float2, double2><<<nb, threads, 0, st>>>(g, L, C, nrhs, in, out)));
}

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

// Block form (4^4 blocks: one workgroup of Bv = 256 threads per block and
// right-hand side).  The block's spinors are staged in LDS once; hops to sites
// of the same block read them there, so memory sees one read of every spinor
// plus the hops across the block faces (a quarter of the sites per direction),
// instead of eight gathers per site that the L2 cannot hold between hops.
template <typename R, typename S, typename Tv, typename To = Tv>
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
  clover_mul<R, S, false>(clov, g.V, I, psi, acc);
  auto fetch = [&](long long J, bool inside, cx<R>* p) {
    if (inside) {
      const int j = (int)(J - base);
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c] = sp[c][j];
    } else {
      load_spinor<R, Tv>(x, g.V, J, p);
    }
  };
  hop_all<R, S>(g, links, s, I, false, fetch, acc);
  store_spinor<R, To>(out + (long long)r * 12 * g.V, g.V, I, acc);
}

// useful flops of one site's D apply: eight hops (project, SU(3) times a half
// spinor, reconstruct and accumulate: 1320), the two packed 6x6 clover blocks
// (504) and the final sum (24)
constexpr double kDiracFlopsPerSite = 1320.0 + 504.0 + 24.0;

}  // namespace

static void dirac_dispatch(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, const void* in, void* out,
                           int threads, hipStream_t st) {
  if (g.Bv == 256 && g.Vc % 16 == 0) {   // block form, slab order over the blocks
    const unsigned nb = xcd_grid(g.Vc, nrhs);
    switch (dt) {
      case DD_F64:
        k_dirac_blk<double, double2, double2><<<nb, 256, 0, st>>>(g, (const double2*)ops.links,
                                                                   (const double2*)ops.clover, nrhs,
                                                                   (const double2*)in, (double2*)out);
        break;
      case DD_F32:
        k_dirac_blk<float, float2, float2><<<nb, 256, 0, st>>>(g, (const float2*)ops.links, (const float2*)ops.clover,
                                                               nrhs, (const float2*)in, (float2*)out);
        break;
      case DD_F16:
        k_dirac_blk<float, __half2, float2><<<nb, 256, 0, st>>>(g, (const __half2*)ops.links,
                                                                (const __half2*)ops.clover, nrhs,
                                                                (const float2*)in, (float2*)out);
        break;
      case DD_BF16:
        k_dirac_blk<float, bf16x2, float2><<<nb, 256, 0, st>>>(g, (const bf16x2*)ops.links, (const bf16x2*)ops.clover,
                                                               nrhs, (const float2*)in, (float2*)out);
        break;
    }
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
    DD_TIMED("k_dirac", st, bytes, flops,
             (k_dirac_blk<double, double2, float2, double2><<<xcd_grid(g.Vc, nrhs), 256, 0, st>>>(g, L, C, nrhs, in,
                                                                                               out)));
    return;
  }
  if (threads != 64 && threads != 128) threads = 256;
  const unsigned nb = xcd_grid((unsigned)((g.V + threads - 1) / threads), nrhs);
  DD_TIMED("k_dirac", st, bytes, flops,
           (k_dirac<double, double2, float2, double2><<<nb, threads, 0, st>>>(g, L, C, nrhs, in, out)));
}

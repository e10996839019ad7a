// Coarse-grid operator apply (Eq. 2 stencil, Sec. 3: "effective links" and
// "clover" blocks of size 2n x 2n).  One workgroup per coarse site; threads
// run over (row, rhs) pairs, and the input vectors of the site and its eight
// neighbours are staged in LDS.  Blocks are column major, so the threads of a
// wave read consecutive rows of one column.
//
//   out(X) = a_self * M(X) xs(X) + a_hop * sum_{d=1..8} D_c(X, d) xh(X + d) + beta * z(X)
//
// with M(X) = D_c(X, 0) (self block) or, for odd sites, the stored inverse of
// the self block.  This covers the full stencil (xs = xh = x), the two halves
// of the even-site Schur complement and the odd-site reconstruction.
#include "dd_internal.h"

namespace {

constexpr int kLdsBytes = 40 * 1024;

template <typename R, typename Sd, typename Tv>
__global__ void __launch_bounds__(256) k_coarse_mv(GeomDev g, int nc, const Sd* __restrict__ Dc,
                                                   const Sd* __restrict__ Minv, int use_inv, int nrhs, int site_begin,
                                                   R a_self, const Tv* __restrict__ xs, R a_hop,
                                                   const Tv* __restrict__ xh, R beta, const Tv* __restrict__ z,
                                                   Tv* __restrict__ out) {
  extern __shared__ unsigned char lds_raw[];
  cx<R>* xsh = reinterpret_cast<cx<R>*>(lds_raw);
  const int X = site_begin + blockIdx.x;
  const long long vstride = (long long)g.Vc * nc;   // rhs stride of a coarse vector
  const int ndir = (a_hop != (R)0) ? 9 : 1;
  const bool has_self = a_self != (R)0;
  int nb[9];
  nb[0] = X;
#pragma unroll
  for (int d = 1; d < 9; ++d) nb[d] = g.blk_nbr[(d - 1) * g.Vc + X] & DD_SLOT_MASK;
  const Sd* Mself = use_inv ? Minv + (long long)(X - g.Vch) * nc * nc : Dc + (long long)X * 9 * nc * nc;
  const Sd* Dx = Dc + (long long)X * 9 * nc * nc;
  // rhs processed in chunks that fit the LDS stage
  int rchunk = kLdsBytes / (int)(9 * nc * sizeof(cx<R>));
  if (rchunk < 1) rchunk = 1;
  for (int r0 = 0; r0 < nrhs; r0 += rchunk) {
    int nr = nrhs - r0 < rchunk ? nrhs - r0 : rchunk;
    __syncthreads();
    for (int e = threadIdx.x; e < ndir * nr * nc; e += blockDim.x) {
      int d = e / (nr * nc), rem = e % (nr * nc), r = rem / nc, c = rem % nc;
      const Tv* src = (d == 0) ? xs : xh;
      cx<R> v = {(R)0, (R)0};
      if (d > 0 || has_self) v = ld<R, Tv>(src + (long long)(r0 + r) * vstride + (long long)nb[d] * nc + c);
      xsh[(d * nr + r) * nc + c] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * nc; e += blockDim.x) {
      int r = e / nc, row = e % nc;
      cx<R> acc_s = {(R)0, (R)0}, acc_h = {(R)0, (R)0};
      if (has_self) {
        const cx<R>* xv = xsh + (0 * nr + r) * nc;
        for (int c = 0; c < nc; ++c) cfma(acc_s, ld<R, Sd>(Mself + (long long)c * nc + row), xv[c]);
      }
      for (int d = 1; d < ndir; ++d) {
        const cx<R>* xv = xsh + (d * nr + r) * nc;
        const Sd* B = Dx + (long long)d * nc * nc;
        for (int c = 0; c < nc; ++c) cfma(acc_h, ld<R, Sd>(B + (long long)c * nc + row), xv[c]);
      }
      cx<R> o = a_self * acc_s + a_hop * acc_h;
      long long oi = (long long)(r0 + r) * vstride + (long long)X * nc + row;
      if (beta != (R)0) o = o + beta * ld<R, Tv>(z + oi);
      st<Tv, R>(out + oi, o);
    }
  }
}

template <typename R, typename Sd, typename Tv>
void mv(const GeomDev& g, int nc, const void* Dc, const void* Minv, int use_inv, int nrhs, int site_begin, int count,
        double a_self, const void* xs, double a_hop, const void* xh, double beta, const void* z, void* out,
        hipStream_t st) {
  if (count <= 0) return;
  k_coarse_mv<R, Sd, Tv><<<(unsigned)count, 256, kLdsBytes, st>>>(
      g, nc, (const Sd*)Dc, (const Sd*)Minv, use_inv, nrhs, site_begin, (R)a_self, (const Tv*)xs, (R)a_hop,
      (const Tv*)xh, (R)beta, (const Tv*)z, (Tv*)out);
}

}  // namespace

void launch_coarse_mv(const GeomDev& g, dd_dtype vt, int nc, const void* Dc, const void* Minv, int use_inv, int nrhs,
                      int site_begin, int count, double a_self, const void* xs, double a_hop, const void* xh,
                      double beta, const void* z, void* out, hipStream_t st) {
  if (vt == DD_F64)
    mv<double, double2, double2>(g, nc, Dc, Minv, use_inv, nrhs, site_begin, count, a_self, xs, a_hop, xh, beta, z, out,
                                 st);
  else
    mv<float, float2, float2>(g, nc, Dc, Minv, use_inv, nrhs, site_begin, count, a_self, xs, a_hop, xh, beta, z, out,
                              st);
}

// canonical coarse vectors [rhs][lex][nc] complex128 <-> packed [rhs][slot][nc]
namespace {
template <typename Tv>
__global__ void k_coarse_perm(GeomDev g, int nc, int nrhs, int to_packed, const void* __restrict__ src,
                              void* __restrict__ dst) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long per = (long long)g.Vc * nc;
  if (e >= per * nrhs) return;
  long long r = e / per, q = e % per;
  int slot = (int)(q / nc), k = (int)(q % nc);
  int bc = g.blk_coord[slot];
  int NB0 = g.L[0] / g.b[0], NB1 = g.L[1] / g.b[1], NB2 = g.L[2] / g.b[2];
  long long lex = (bc & 255) + NB0 * (((bc >> 8) & 255) + NB1 * (((bc >> 16) & 255) + (long long)NB2 * ((bc >> 24) & 255)));
  long long ip = r * per + (long long)slot * nc + k, ic = r * per + lex * nc + k;
  if (to_packed) {
    double2 v = ((const double2*)src)[ic];
    st<Tv, double>((Tv*)dst + ip, cx<double>{v.x, v.y});
  } else {
    cx<double> v = ld<double, Tv>((const Tv*)src + ip);
    ((double2*)dst)[ic] = make_double2(v.re, v.im);
  }
}
}  // namespace

void launch_coarse_perm(const GeomDev& g, dd_dtype vt, int nc, int nrhs, int to_packed, const void* src, void* dst,
                        hipStream_t st) {
  long long n = (long long)g.Vc * nc * nrhs;
  unsigned nb = (unsigned)((n + 255) / 256);
  if (vt == DD_F64)
    k_coarse_perm<double2><<<nb, 256, 0, st>>>(g, nc, nrhs, to_packed, src, dst);
  else
    k_coarse_perm<float2><<<nb, 256, 0, st>>>(g, nc, nrhs, to_packed, src, dst);
}

// Coarse-grid operator apply (Eq. 2 stencil, Sec. 3: "effective links" and
// "clover" blocks of size 2n x 2n).  Blocks are column major, so the lanes of
// a wave read consecutive rows of one column.
//
//   out(X) = a_self * M(X) xs(X) + a_hop * sum_{d=1..8} D_c(X, d) xh(X + d) + beta * z(X)
//
// with M(X) = D_c(X, 0) (self block) or, for odd sites, the stored inverse of
// the self block.  This covers the full stencil (xs = xh = x), the two halves
// of the even-site Schur complement and the odd-site reconstruction.
#include <type_traits>

#include "dd_internal.h"
#include "ktimer.h"

namespace {

// One wave per coarse site, lane = row of the 2n x 2n blocks (2n <= 64); NR
// right-hand sides are accumulated per lane.  The input of the site / its
// neighbour for the current direction is staged in LDS as [col][rhs], so each
// lane streams one column of the block (coalesced over the wave) against an
// LDS broadcast of the inputs: every block element is read once per apply.
constexpr int kSitesPerWG = 4;

template <typename R, typename Sd, typename Tv, int NR>
__global__ void __launch_bounds__(64 * kSitesPerWG) k_coarse_mv(GeomDev g, int nc, const Sd* __restrict__ Dc,
                                                              const Sd* __restrict__ Minv, int use_inv, int nrhs,
                                                              int site_begin, int count, R a_self,
                                                              const Tv* __restrict__ xs, R a_hop,
                                                              const Tv* __restrict__ xh, R beta,
                                                              const Tv* __restrict__ z, Tv* __restrict__ out,
                                                              Gate gt) {
  if (gate_closed(gt)) return;
  __shared__ cx<R> xsh[kSitesPerWG][64][NR];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int local = blockIdx.x * kSitesPerWG + w;
  const bool site_ok = local < count;
  const int X = site_begin + (site_ok ? local : 0);
  const long long vstride = (long long)g.Vc * nc;   // rhs stride of a coarse vector
  const bool has_self = a_self != (R)0, has_hop = a_hop != (R)0;
  const bool row_ok = site_ok && lane < nc;
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = nrhs - r0 < NR ? nrhs - r0 : NR;
    cx<R> acc_s[NR], acc_h[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc_s[r] = acc_h[r] = {(R)0, (R)0};
    for (int d = has_self ? 0 : 1; d < (has_hop ? 9 : 1); ++d) {
      const int Y = d == 0 ? X : (g.blk_nbr[(d - 1) * g.Vc + X] & DD_SLOT_MASK);
      const Tv* src = d == 0 ? xs : xh;
      __syncthreads();
      if (row_ok)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) xsh[w][lane][r] = ld<R, Tv>(src + (long long)(r0 + r) * vstride + (long long)Y * nc + lane);
      __syncthreads();
      if (row_ok) {
        const Sd* B = d == 0 ? (use_inv ? Minv + (long long)(X - g.Vch) * nc * nc : Dc + (long long)X * 9 * nc * nc)
                             : Dc + ((long long)X * 9 + d) * nc * nc;
        cx<R> acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = {(R)0, (R)0};
        for (int c = 0; c < nc; ++c) {
          cx<R> m = ld<R, Sd>(B + (long long)c * nc + lane);
#pragma unroll
          for (int r = 0; r < NR; ++r)
            if (r < nr) cfma(acc[r], m, xsh[w][c][r]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (d == 0) acc_s[r] = acc[r];
          else acc_h[r] = acc_h[r] + acc[r];
        }
      }
    }
    if (row_ok)
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nr) {
          long long oi = (long long)(r0 + r) * vstride + (long long)X * nc + lane;
          cx<R> o = a_self * acc_s[r] + a_hop * acc_h[r];
          if (beta != (R)0) o = o + beta * ld<R, Tv>(z + oi);
          st<Tv, R>(out + oi, o);
        }
  }
}

// FP32 matrix-core form.  For one coarse site and one direction the stencil
// term is a complex GEMM Y (2n x NRHS) += B (2n x 2n) X (2n x NRHS).  With
// B = Br + i Bi, X = Xr + i Xi it is computed as four real 16x16x4 MFMA
// products per (16-row tile, 4-deep k step): tile C0 collects Y_r = Br Xr - Bi Xi
// and tile C1 collects Y_i = Br Xi + Bi Xr, with the right-hand side as the
// column index of both tiles, so each lane ends with the real and imaginary
// part of the same (row, rhs).  Lane layout of v_mfma_f32_16x16x4f32: A[i][k]
// at lane i + 16k, B[k][j] at lane j + 16k, D[i][j] at lane j + 16(i/4), value
// i % 4.  One wave per site, up to 16 right-hand sides per pass, 2n <= 48.
// Matrix-core order of one NC x NC block (the FP32 and half copies the FP32
// apply reads).  Element (row, col) lies in row tile t = row / 16 (RT = min(16,
// NC - 16 t) rows) and k-step ks = col / 4 (lane group lk = col % 4); P
// consecutive k-steps form a group q = ks / P.  Within a tile the order is
// [q][lk][li][e]: lane (li, lk) of the MFMA operand reads its P k-steps of row
// 16 t + li with one load of P elements, and a wave reads one contiguous stretch.
// No padding: a block still holds NC * NC elements.
__host__ __device__ inline long long tiled_off(int row, int col, int NC, int P) {
  const int t = row >> 4, li = row & 15, RT = NC - 16 * t < 16 ? NC - 16 * t : 16;
  const int ks = col >> 2, lk = col & 3, q = ks / P, e = ks % P;
  return (long long)16 * t * NC + ((long long)(q * 4 + lk) * RT + li) * P + e;
}
// P: the largest power of two k-steps per load (at most 16 bytes) that divides NC / 4
__host__ __device__ constexpr int tile_group(int NC, int elem_bytes) {
  return ((NC / 4) % (16 / elem_bytes) == 0) ? 16 / elem_bytes : (((NC / 4) % 2 == 0 && 16 / elem_bytes >= 2) ? 2 : 1);
}

// FP64 column-major blocks -> FP32 blocks in matrix-core order
__global__ void k_tile_f32(const double2* __restrict__ src, float2* __restrict__ dst, long long nblk, int NC) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)NC * NC;
  if (i >= nblk * per) return;
  const long long b = i / per, w = i % per;
  const int row = (int)(w % NC), col = (int)(w / NC);
  const double2 v = src[i];
  dst[b * per + tiled_off(row, col, NC, tile_group(NC, 8))] = make_float2((float)v.x, (float)v.y);
}
// FP32 matrix-core blocks -> half matrix-core blocks (rounded from the FP32 values)
template <typename H>
__global__ void k_tile_half(const float2* __restrict__ src, H* __restrict__ dst, long long nblk, int NC) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)NC * NC;
  if (i >= nblk * per) return;
  const long long b = i / per, w = i % per;
  const int row = (int)(w % NC), col = (int)(w / NC);
  const float2 v = src[b * per + tiled_off(row, col, NC, tile_group(NC, 8))];
  H* d = dst + b * per + tiled_off(row, col, NC, tile_group(NC, 4));
  if constexpr (sizeof(H) == 4 && std::is_same<H, __half2>::value) {
    *d = __floats2half2_rn(v.x, v.y);
  } else {
    d->u = f32_to_bf16_bits(v.x) | (f32_to_bf16_bits(v.y) << 16);
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaMaxNc = 48;

// NC = 2n (a multiple of 4, at most 48).  A workgroup takes S coarse sites with
// MT = ceil(NC / 16) waves per site, one per 16-row tile of the NC rows: each
// wave streams its rows of the site's 9 (or 1, or 8) blocks into registers,
// while the MT waves of the site stage sc * x(Y) for 16 right-hand sides (zero
// weight past nrhs) in LDS with loads along the columns, one barrier per
// direction (double-buffered staging).  Complex products use three real MFMAs
// (Gauss): with A = a + ib and x = c + id,
//   k1 += a (c + d),  k2 += (a + b)(-d),  k3 += (b - a) c,
//   Re(A x) = k1 + k2,  Im(A x) = k1 + k3.
// Site groups are dealt to the XCDs in contiguous eighths, so the neighbours'
// x of one range come from the same L2.
template <int NC, int S, typename Sd>
__global__ void __launch_bounds__(64 * S * ((NC + 15) / 16)) k_coarse_mfma(
    GeomDev g, const Sd* __restrict__ Dc, const Sd* __restrict__ Minv, int use_inv, int nrhs, int site_begin,
    int count, float a_self, const float2* __restrict__ xs, float a_hop, const float2* __restrict__ xh, float beta,
    const float2* __restrict__ z, float2* __restrict__ out, Gate gt) {
  if (gate_closed(gt)) return;
  constexpr int MT = (NC + 15) / 16, KS = NC / 4, XP = 17;
  constexpr int P = tile_group(NC, (int)sizeof(Sd));
  struct alignas(P * sizeof(Sd)) Pack {
    Sd v[P];
  };
  __shared__ float2 xsh[S][2][NC][XP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s_in = wv / MT, t = wv % MT, tid_site = threadIdx.x - 64 * MT * s_in;
  const int ngroups = (count + S - 1) / S, per_x = (ngroups + 7) / 8;
  const int group = (blockIdx.x & 7) * per_x + (blockIdx.x >> 3);
  if (group >= ngroups) return;   // uniform per workgroup
  const int local = group * S + s_in;
  const bool site_ok = local < count;   // S > 1: the last group may be short (its waves still reach the barriers)
  const int X = site_begin + (site_ok ? local : 0);
  const int RT = NC - 16 * t < 16 ? NC - 16 * t : 16;
  const long long vstride = (long long)g.Vc * NC;
  const bool has_self = a_self != 0.f, has_hop = a_hop != 0.f;
  const int li = lane & 15, lk = lane >> 4;
  const bool row_ok = li < RT;
  int buf = 0;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
    const bool rhs_ok = li < nr;
    f32x4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = k1, k3 = k1;
    for (int d = has_self ? 0 : 1; d < (has_hop ? 9 : 1); ++d) {
      const int Y = d == 0 ? X : (g.blk_nbr[(d - 1) * g.Vc + X] & DD_SLOT_MASK);
      const float2* src = d == 0 ? xs : xh;
      const float sc = d == 0 ? a_self : a_hop;
      const Sd* B = d == 0 ? (use_inv ? Minv + (long long)(X - g.Vch) * NC * NC : Dc + (long long)X * 9 * NC * NC)
                           : Dc + ((long long)X * 9 + d) * NC * NC;
      const Sd* Bt = B + (long long)16 * t * NC;
      // x(Y) first (consecutive threads of the site take consecutive columns; the
      // loads are clamped into the nr right-hand sides), then this wave's rows of
      // the block (rows 16t + li, columns 4 ks + lk, P k-steps per load, see
      // tiled_off), so the staging waits for the x loads only
      constexpr int XI = (16 * NC + 64 * MT - 1) / (64 * MT);
      const int nx = nr * NC;
      float2 xv[XI];
#pragma unroll
      for (int i = 0; i < XI; ++i) {
        const int e = tid_site + 64 * MT * i, ec = e < nx ? e : nx - 1;
        const int r = ec / NC, col = ec - r * NC;
        xv[i] = src[(long long)(r0 + r) * vstride + (long long)Y * NC + col];
      }
      Pack pk[KS / P];
#pragma unroll
      for (int q = 0; q < KS / P; ++q)
        pk[q] = *reinterpret_cast<const Pack*>(Bt + ((long long)(q * 4 + lk) * RT + (row_ok ? li : 0)) * P);
      // stage sc * x(Y) as [col][rhs]
#pragma unroll
      for (int i = 0; i < XI; ++i) {
        const int e = tid_site + 64 * MT * i;
        if (e < nx) {
          const int r = e / NC, col = e - r * NC;
          xsh[s_in][buf][col][r] = make_float2(sc * xv[i].x, sc * xv[i].y);
        }
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const cx<float> m = row_ok ? ld<float, Sd>(&pk[ks / P].v[ks % P]) : cx<float>{0.f, 0.f};
        const float2 xb = xsh[s_in][buf][4 * ks + lk][li];
        const float c = rhs_ok ? xb.x : 0.f, dd = rhs_ok ? xb.y : 0.f;
        k1 = __builtin_amdgcn_mfma_f32_16x16x4f32(m.re, c + dd, k1, 0, 0, 0);
        k2 = __builtin_amdgcn_mfma_f32_16x16x4f32(m.re + m.im, -dd, k2, 0, 0, 0);
        k3 = __builtin_amdgcn_mfma_f32_16x16x4f32(m.im - m.re, c, k3, 0, 0, 0);
      }
      buf ^= 1;
    }
    if (site_ok && rhs_ok) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + 4 * lk + v;
        if (row < NC) {
          long long oi = (long long)(r0 + li) * vstride + (long long)X * NC + row;
          float2 o = make_float2(k1[v] + k2[v], k1[v] + k3[v]);
          if (beta != 0.f) {
            float2 zz = z[oi];
            o.x += beta * zz.x;
            o.y += beta * zz.y;
          }
          out[oi] = o;
        }
      }
    }
  }
}

// Half-precision matrix-core form (opt-in, half-precision blocks only): the
// blocks feed 16x16x16 FP16 / BF16 MFMAs directly and sc * x(Y) is rounded to
// the same type when staged; products accumulate in FP32 (four real MFMAs per
// complex product: k1 = a c, k2 = b d, k3 = a d, k4 = b c).  MFMA K-slot
// (lk, v) of K-step s takes column 4 (4 s + v) + lk, so every lane's four A
// values sit at one (row, lk) of the tiled block layout (see tiled_off);
// columns past NC are zero on both sides.
typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));
typedef short b16x4 __attribute__((ext_vector_type(4)));

template <typename Sd> struct HalfOp;
template <> struct HalfOp<__half2> {
  typedef h16x4 vec;
  typedef _Float16 elem;
  __device__ static elem from_f32(float f) { return (_Float16)f; }
  __device__ static void split(const __half2& v, elem& re, elem& im) {
    const __half2_raw r = v;
    re = __builtin_bit_cast(_Float16, r.x);
    im = __builtin_bit_cast(_Float16, r.y);
  }
  __device__ static f32x4 mfma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};
template <> struct HalfOp<bf16x2> {
  typedef b16x4 vec;
  typedef short elem;
  __device__ static elem from_f32(float f) { return (short)f32_to_bf16_bits(f); }
  __device__ static void split(const bf16x2& v, elem& re, elem& im) {
    re = (short)(v.u & 0xffffu);
    im = (short)(v.u >> 16);
  }
  __device__ static f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

// Two directions per barrier phase: the loads of both directions' blocks and
// inputs are in flight together (five phases for the nine-block stencil
// instead of nine), which matters because one apply is a single round of
// workgroups whose time is the chain of load latencies.  The directions are
// still accumulated in order, so the result is that of one direction per phase.
// With both directions' operands live the compiler would take about 164
// registers (two waves per SIMD); the register budget is capped at four waves
// per SIMD instead (the BF16 form then spills 12 bytes per lane).
template <int NC, int S, typename Sd>
__global__ void __launch_bounds__(64 * S * ((NC + 15) / 16)) __attribute__((amdgpu_waves_per_eu(4))) k_coarse_mfma_h(
    GeomDev g, const Sd* __restrict__ Dc, const Sd* __restrict__ Minv, int use_inv, int nrhs, int site_begin,
    int count, float a_self, const float2* __restrict__ xs, float a_hop, const float2* __restrict__ xh, float beta,
    const float2* __restrict__ z, float2* __restrict__ out, Gate gt) {
  if (gate_closed(gt)) return;
  typedef HalfOp<Sd> H;
  typedef typename H::vec vec;
  typedef typename H::elem elem;
  constexpr int MT = (NC + 15) / 16, KS = NC / 4, NS = (KS + 3) / 4, DP = 2;
  constexpr int P = tile_group(NC, (int)sizeof(Sd));
  constexpr int XI = (16 * NC + 64 * MT - 1) / (64 * MT);
  // staged x: [site][buffer][direction of the phase][s][lk][rhs][v], real and imaginary parts
  __shared__ alignas(16) elem xc[S][2][DP][NS][4][16][4];
  __shared__ alignas(16) elem xd[S][2][DP][NS][4][16][4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s_in = wv / MT, t = wv % MT, tid_site = threadIdx.x - 64 * MT * s_in;
  const int ngroups = (count + S - 1) / S, per_x = (ngroups + 7) / 8;
  const int group = (blockIdx.x & 7) * per_x + (blockIdx.x >> 3);
  if (group >= ngroups) return;   // uniform per workgroup
  const int local = group * S + s_in;
  const bool site_ok = local < count;
  // the site is the same on every lane of a wave: keep it (and the block and
  // neighbour addresses derived from it) in scalar registers
  const int X = __builtin_amdgcn_readfirstlane(site_begin + (site_ok ? local : 0));
  const int RT = NC - 16 * t < 16 ? NC - 16 * t : 16;
  const long long vstride = (long long)g.Vc * NC;
  const bool has_self = a_self != 0.f, has_hop = a_hop != 0.f;
  const int d_begin = has_self ? 0 : 1, d_end = has_hop ? 9 : 1;
  const int li = lane & 15, lk = lane >> 4;
  const bool row_ok = li < RT;
  // K-slots past NC stay zero in every buffer
  {
    elem* pc = &xc[s_in][0][0][0][0][0][0];
    elem* pd = &xd[s_in][0][0][0][0][0][0];
    for (int e = tid_site; e < 2 * DP * NS * 4 * 16 * 4; e += 64 * MT) {
      pc[e] = H::from_f32(0.f);
      pd[e] = H::from_f32(0.f);
    }
  }
  __syncthreads();
  int buf = 0;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
    const bool rhs_ok = li < nr;
    const int nx = nr * NC;
    f32x4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = k1, k3 = k1, k4 = k1;
    for (int d0 = d_begin; d0 < d_end; d0 += DP) {
      const int nd = d_end - d0 < DP ? d_end - d0 : DP;   // uniform
      float2 xv[DP][XI];
      Sd av[DP][NS][4];
#pragma unroll
      for (int q = 0; q < DP; ++q) {
        if (q >= nd) break;
        const int d = d0 + q;
        const int Y = d == 0 ? X : __builtin_amdgcn_readfirstlane(g.blk_nbr[(d - 1) * g.Vc + X] & DD_SLOT_MASK);
        const float2* xsrc = (d == 0 ? xs : xh) + (long long)r0 * vstride + (long long)Y * NC;
        const Sd* B = d == 0 ? (use_inv ? Minv + (long long)(X - g.Vch) * NC * NC : Dc + (long long)X * 9 * NC * NC)
                             : Dc + ((long long)X * 9 + d) * NC * NC;
        const Sd* Bt = B + 16 * t * NC;
#pragma unroll
        for (int i = 0; i < XI; ++i) {
          const int e = tid_site + 64 * MT * i, ec = e < nx ? e : nx - 1;
          const int r = ec / NC, col = ec - r * NC;
          xv[q][i] = xsrc[(unsigned)(r * (int)vstride + col)];   // < 16 * Vc * NC elements
        }
        // this wave's rows: K-step s, slot v -> tiled column group ks = 4 s + v at this lane's lk
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ks = 4 * st + v;
            if (ks < KS) av[q][st][v] = Bt[(unsigned)((((ks / P) * 4 + lk) * RT + (row_ok ? li : 0)) * P + ks % P)];
          }
      }
#pragma unroll
      for (int q = 0; q < DP; ++q) {
        if (q >= nd) break;
        const float sc = d0 + q == 0 ? a_self : a_hop;
#pragma unroll
        for (int i = 0; i < XI; ++i) {
          const int e = tid_site + 64 * MT * i;
          if (e < nx) {
            const int r = e / NC, col = e - r * NC;
            const int ks = col >> 2, cl = col & 3;
            xc[s_in][buf][q][ks >> 2][cl][r][ks & 3] = H::from_f32(sc * xv[q][i].x);
            xd[s_in][buf][q][ks >> 2][cl][r][ks & 3] = H::from_f32(sc * xv[q][i].y);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < DP; ++q) {
        if (q >= nd) break;
#pragma unroll
        for (int st = 0; st < NS; ++st) {
          vec a, b;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            elem re = H::from_f32(0.f), im = H::from_f32(0.f);
            if (4 * st + v < KS && row_ok) H::split(av[q][st][v], re, im);
            a[v] = re;
            b[v] = im;
          }
          vec c = *reinterpret_cast<const vec*>(&xc[s_in][buf][q][st][lk][li][0]);
          vec dd = *reinterpret_cast<const vec*>(&xd[s_in][buf][q][st][lk][li][0]);
          if (!rhs_ok) {
            c = vec{};
            dd = vec{};
          }
          k1 = H::mfma(a, c, k1);
          k2 = H::mfma(b, dd, k2);
          k3 = H::mfma(a, dd, k3);
          k4 = H::mfma(b, c, k4);
        }
      }
      buf ^= 1;
    }
    if (site_ok && rhs_ok) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + 4 * lk + v;
        if (row < NC) {
          long long oi = (long long)(r0 + li) * vstride + (long long)X * NC + row;
          float2 o = make_float2(k1[v] - k2[v], k3[v] + k4[v]);
          if (beta != 0.f) {
            float2 zz = z[oi];
            o.x += beta * zz.x;
            o.y += beta * zz.y;
          }
          out[oi] = o;
        }
      }
    }
  }
}

typedef void (*MfmaFn)(GeomDev, const void*, const void*, int, int, int, int, float, const float2*, float,
                       const float2*, float, const float2*, float2*, Gate);

// spw: target waves per workgroup; sites per workgroup S = max(1, spw / MT), at most 4
template <int NC, typename Sd, bool HM = false>
MfmaFn mfma_spw(int spw, unsigned count, dim3& grid, dim3& blk) {
  constexpr int MT = (NC + 15) / 16;
  int S = spw / MT;
  MfmaFn fn;
  if (S >= 4) S = 4;
  else if (S >= 2) S = 2;
  else S = 1;
  if constexpr (HM) {
    fn = S == 4 ? (MfmaFn)k_coarse_mfma_h<NC, 4, Sd> : S == 2 ? (MfmaFn)k_coarse_mfma_h<NC, 2, Sd>
                                                              : (MfmaFn)k_coarse_mfma_h<NC, 1, Sd>;
  } else {
    fn = S == 4 ? (MfmaFn)k_coarse_mfma<NC, 4, Sd> : S == 2 ? (MfmaFn)k_coarse_mfma<NC, 2, Sd>
                                                            : (MfmaFn)k_coarse_mfma<NC, 1, Sd>;
  }
  const unsigned per_x = ((count + S - 1) / S + 7) / 8;   // see k_coarse_mfma
  grid = dim3(8 * per_x);
  blk = dim3(64 * S * MT);
  return fn;
}

template <typename Sd, bool HM = false>
MfmaFn mfma_pick(int nc, int spw, unsigned count, dim3& grid, dim3& blk) {
  switch (nc) {
    case 12: return mfma_spw<12, Sd, HM>(spw, count, grid, blk);
    case 16: return mfma_spw<16, Sd, HM>(spw, count, grid, blk);
    case 24: return mfma_spw<24, Sd, HM>(spw, count, grid, blk);
    case 32: return mfma_spw<32, Sd, HM>(spw, count, grid, blk);
    case 40: return mfma_spw<40, Sd, HM>(spw, count, grid, blk);
    default: return mfma_spw<48, Sd, HM>(spw, count, grid, blk);
  }
}

template <typename R, typename Sd, typename Tv>
void mv(const GeomDev& g, int nc, const void* Dc, const void* Minv, int use_inv, int nrhs, int site_begin, int count,
        double a_self, const void* xs, double a_hop, const void* xh, double beta, const void* z, void* out,
        hipStream_t st, int spw, dd_dtype bt, bool hm) {
  if (count <= 0) return;
  const int nblocks_read = (a_self != 0.0 ? 1 : 0) + (a_hop != 0.0 ? 8 : 0);
  const double bytes = (double)count * nblocks_read * nc * nc * sizeof(Sd) +
                       (double)count * nc * nrhs * sizeof(Tv) * (2 + (beta != 0.0 ? 1 : 0));
  const double flops = 8.0 * count * nblocks_read * nc * nc * nrhs;
  const unsigned nb = (unsigned)((count + kSitesPerWG - 1) / kSitesPerWG);
  const dim3 blk(64 * kSitesPerWG);
#define DD_MV(NRV)                                                                                                 \
  DD_TIMED("k_coarse_mv", st, bytes, flops,                                                                        \
           (k_coarse_mv<R, Sd, Tv, NRV><<<nb, blk, 0, st>>>(g, nc, (const Sd*)Dc, (const Sd*)Minv, use_inv, nrhs,   \
                                                             site_begin, count, (R)a_self, (const Tv*)xs, (R)a_hop, \
                                                             (const Tv*)xh, (R)beta, (const Tv*)z, (Tv*)out, \
                                                             current_gate())))
  if (sizeof(R) == 4 && nc <= kMfmaMaxNc) {
    dim3 grid, wg;
    MfmaFn fn = bt == DD_F16    ? (hm ? mfma_pick<__half2, true>(nc, spw, count, grid, wg)
                                      : mfma_pick<__half2>(nc, spw, count, grid, wg))
                : bt == DD_BF16 ? (hm ? mfma_pick<bf16x2, true>(nc, spw, count, grid, wg)
                                      : mfma_pick<bf16x2>(nc, spw, count, grid, wg))
                                : mfma_pick<float2>(nc, spw, count, grid, wg);
    const double hb = bt == DD_F32 ? 1.0 : 0.5;   // half-precision blocks stream half the bytes
    DD_TIMED("k_coarse_mfma", st, bytes - (1.0 - hb) * (double)count * nblocks_read * nc * nc * sizeof(Sd), flops,
             (fn<<<grid, wg, 0, st>>>(g, Dc, Minv, use_inv, nrhs, site_begin, count, (float)a_self, (const float2*)xs,
                                      (float)a_hop, (const float2*)xh, (float)beta, (const float2*)z, (float2*)out,
                                      current_gate())));
  } else if (nrhs == 1) DD_MV(1);
  else if (nrhs <= 4) DD_MV(4);
  else DD_MV(12);
#undef DD_MV
}

}  // namespace

void launch_coarse_tile(int nc, const double2* src64, long long nblk, float2* dst32, dd_dtype half, void* dsth,
                        hipStream_t st) {
  const long long n = nblk * nc * nc;
  const unsigned nb = (unsigned)((n + 255) / 256);
  k_tile_f32<<<nb, 256, 0, st>>>(src64, dst32, nblk, nc);
  if (half == DD_F16) k_tile_half<__half2><<<nb, 256, 0, st>>>(dst32, (__half2*)dsth, nblk, nc);
  if (half == DD_BF16) k_tile_half<bf16x2><<<nb, 256, 0, st>>>(dst32, (bf16x2*)dsth, nblk, nc);
}

void launch_coarse_mv(const GeomDev& g, dd_dtype vt, int nc, const void* Dc, const void* Minv, int use_inv, int nrhs,
                      int site_begin, int count, double a_self, const void* xs, double a_hop, const void* xh,
                      double beta, const void* z, void* out, hipStream_t st, int spw, dd_dtype bt, bool hm) {
  if (vt == DD_F64)
    mv<double, double2, double2>(g, nc, Dc, Minv, use_inv, nrhs, site_begin, count, a_self, xs, a_hop, xh, beta, z, out,
                                 st, spw, DD_F64, false);
  else
    mv<float, float2, float2>(g, nc, Dc, Minv, use_inv, nrhs, site_begin, count, a_self, xs, a_hop, xh, beta, z, out,
                              st, spw, bt, hm && (bt == DD_F16 || bt == DD_BF16));
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

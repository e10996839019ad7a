// Third multigrid level (the paper runs two and notes that the coarse solver
// may itself be a multigrid method, Sec. 1, Sec. 2): the construction of
// Eqs. (1)-(4) applied once more, to the coarse operator D_c of Eq. (2).
// Level-2 aggregates are blocks of 2^4 coarse sites; a coarse vector's
// chirality s is its components s*n .. s*n + n - 1.  The level-2 test vectors
// give P2 [X3][s][i][l*n + c] (l: position of the coarse site in its block, c:
// component within chirality s), orthonormalised per (X3, s); R2 = P2^dag and
// D3 = P2^dag D_c P2 per stored direction, in the coarse blocks' layout.
#include "ktimer.h"
#include "dd_internal.h"

namespace {

constexpr int kL = 16;   // coarse sites per level-2 aggregate

// modified Gram-Schmidt (two projection sweeps, vectors in order) of the n2
// vectors of one (X3, s) set, gathered from the level-2 test vectors
// tv [n2][Vc][2n] (slot order) into their place in P2 and worked there (a set
// is at most 24 x 384 entries, read through the cache); one workgroup per set
__global__ void __launch_bounds__(256) k_gs2(int Vc, int n, int n2, const int* __restrict__ slot_of,
                                             const double2* __restrict__ tv, double2* __restrict__ P2, int* bad) {
  __shared__ double red[2][4];
  const int X3 = blockIdx.x >> 1, s = blockIdx.x & 1, K = kL * n;
  double2* g = P2 + (long long)blockIdx.x * n2 * K;
  for (int e = threadIdx.x; e < n2 * K; e += blockDim.x) {
    const int i = e / K, k = e - i * K, l = k / n, c = k - l * n;
    g[e] = tv[((long long)i * Vc + slot_of[X3 * kL + l]) * 2 * n + s * n + c];
  }
  __threadfence_block();
  __syncthreads();
  auto dot = [&](int a, int b) {   // <g_a, g_b>, every thread gets it
    double re = 0.0, im = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const double2 x = g[a * K + k], y = g[b * K + k];
      re += x.x * y.x + x.y * y.y;
      im += x.x * y.y - x.y * y.x;
    }
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();   // the previous reduction's reads of red are done
    if ((threadIdx.x & 63) == 0) {
      red[0][w] = re;
      red[1][w] = im;
    }
    __syncthreads();
    re = im = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      re += red[0][q];
      im += red[1][q];
    }
    return double2{re, im};
  };
  for (int i = 0; i < n2; ++i) {
    const double nrm0 = sqrt(dot(i, i).x);
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < i; ++j) {
        const double2 d = dot(j, i);
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
          const double2 q = g[j * K + k];
          double2 v = g[i * K + k];
          v.x -= d.x * q.x - d.y * q.y;
          v.y -= d.x * q.y + d.y * q.x;
          g[i * K + k] = v;
        }
        __threadfence_block();
        __syncthreads();
      }
    const double nrm = sqrt(dot(i, i).x);
    if (!(nrm > 1e-12 * nrm0)) {
      if (threadIdx.x == 0) atomicMax(bad, (int)blockIdx.x);
      return;   // uniform: every thread saw the same norms
    }
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      double2 v = g[i * K + k];
      v.x /= nrm;
      v.y /= nrm;
      g[i * K + k] = v;
    }
    __threadfence_block();
    __syncthreads();
  }
}

// out[r][X3][s*n2 + i] = sum_{l, c} conj(P2[X3][s][i][l*n + c]) v[r][slot_of[X3][l]][s*n + c]
// one workgroup per (X3, r), 16 lanes per output (one workgroup looping over the right-hand
// sides with P2 in registers was slower: too few workgroups for the level-3 lattice)
template <typename Tp, typename Tv>
__global__ void __launch_bounds__(256) k_restrict2(int Vc, int Vc3, int n, int n2, const int* __restrict__ slot_of,
                                                   const Tp* __restrict__ P2, const Tv* __restrict__ v,
                                                   Tv* __restrict__ out) {
  const int X3 = blockIdx.x, r = blockIdx.y, K = kL * n;
  const int lane16 = threadIdx.x & 15;
  for (int o = threadIdx.x >> 4; o < 2 * n2; o += blockDim.x >> 4) {
    const int s = o / n2, i = o - s * n2;
    const Tp* p = P2 + ((long long)(X3 * 2 + s) * n2 + i) * K;
    double re = 0.0, im = 0.0;
    for (int k = lane16; k < K; k += 16) {
      const int l = k / n, c = k - l * n;
      const Tp a = p[k];
      const Tv b = v[((long long)r * Vc + slot_of[X3 * kL + l]) * 2 * n + s * n + c];
      re += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
      im += (double)a.x * (double)b.y - (double)a.y * (double)b.x;
    }
    for (int off = 8; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 16);
      im += __shfl_xor(im, off, 16);
    }
    if (lane16 == 0) {
      Tv res;
      res.x = (decltype(res.x))re;
      res.y = (decltype(res.y))im;
      out[((long long)r * Vc3 + X3) * 2 * n2 + o] = res;
    }
  }
}

constexpr int kMaxPer = 24;   // n2 <= 24

// out[r][x][s*n + c] = sum_i P2[X3(x)][s][i][l(x)*n + c] y[r][X3(x)][s*n2 + i]; one thread per (x, component),
// its n2 entries of P2 in registers across the right-hand sides
template <typename Tp, typename Tv>
__global__ void __launch_bounds__(256) k_prolong2(int Vc, int Vc3, int n, int n2, const int* __restrict__ l3_of,
                                                  const int* __restrict__ loc_of, const Tp* __restrict__ P2,
                                                  const Tv* __restrict__ y, Tv* __restrict__ out, int nrhs) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)Vc * 2 * n;
  if (e >= per) return;
  const int x = (int)(e / (2 * n)), comp = (int)(e - (long long)x * 2 * n);
  const int s = comp / n, c = comp - s * n, X3 = l3_of[x], l = loc_of[x], K = kL * n;
  const Tp* p = P2 + ((long long)(X3 * 2 + s) * n2) * K + l * n + c;
  Tp pi[kMaxPer];
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) pi[i] = i < n2 ? p[(long long)i * K] : Tp{};
  for (int r = 0; r < nrhs; ++r) {
    const Tv* yy = y + ((long long)r * Vc3 + X3) * 2 * n2 + s * n2;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      if (i < n2) {   // predicated, not a break: pi stays in registers
        const Tp a = pi[i];
        const Tv b = yy[i];
        re += (double)a.x * (double)b.x - (double)a.y * (double)b.y;
        im += (double)a.x * (double)b.y + (double)a.y * (double)b.x;
      }
    }
    Tv res;
    res.x = (decltype(res.x))re;
    res.y = (decltype(res.y))im;
    out[(long long)r * per + e] = res;
  }
}

// D3[X3][d3] (column-major 2n2 x 2n2 block): sum over the coarse sites x of X3
// and stored directions dd with crossing(x, dd) == d3 of P2(x)^dag D_c(x, dd) P2(x + dd).
// One workgroup per (X3, d3); per pair T = D_c(x, dd) P2(y)^T is staged in LDS.
__global__ void __launch_bounds__(256) k_galerkin3(GeomDev g2, int n, int n2, const int* __restrict__ slot_of,
                                                   const int* __restrict__ l3_of, const int* __restrict__ loc_of,
                                                   const double2* __restrict__ Dc, const double2* __restrict__ P2,
                                                   double2* __restrict__ D3) {
  extern __shared__ double2 T[];   // [2n][2 n2]
  const int X3 = blockIdx.x / 9, d3 = blockIdx.x % 9, nc = 2 * n, nc3 = 2 * n2, K = kL * n;
  const int Vc = g2.Vc;
  constexpr int kQ = 9;            // outputs a*nc3 + b = threadIdx.x + 256 q, q < kQ (nc3 <= 48)
  double2 acc[kQ] = {};
  for (int l = 0; l < kL; ++l) {
    const int x = slot_of[X3 * kL + l];
    const int lc[4] = {l & 1, (l >> 1) & 1, (l >> 2) & 1, (l >> 3) & 1};
    for (int dd = 0; dd < 9; ++dd) {
      int cross = 0;
      if (dd) {
        const int mu = (dd - 1) & 3, sg = dd <= 4 ? 1 : -1;
        const int v = lc[mu] + sg;
        cross = (v < 0 || v > 1) ? dd : 0;
      }
      if (cross != d3) continue;   // uniform over the workgroup
      const int y = dd == 0 ? x : (g2.blk_nbr[(dd - 1) * Vc + x] & DD_SLOT_MASK);
      const int Y3 = l3_of[y], ly = loc_of[y];
      const double2* B = Dc + ((long long)x * 9 + dd) * nc * nc;   // element (row c, col e) at e * nc + c
      __syncthreads();   // the previous pair's reads of T are done
      for (int t = threadIdx.x; t < nc * nc3; t += blockDim.x) {
        const int c = t / nc3, b = t - c * nc3, sb = b / n2, ib = b - sb * n2;
        const double2* p = P2 + ((long long)(Y3 * 2 + sb) * n2 + ib) * K + ly * n;
        double re = 0.0, im = 0.0;
        for (int e = 0; e < n; ++e) {
          const double2 m = B[(long long)(sb * n + e) * nc + c], q = p[e];
          re += m.x * q.x - m.y * q.y;
          im += m.x * q.y + m.y * q.x;
        }
        T[t] = double2{re, im};
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int o = threadIdx.x + 256 * q;
        if (o >= nc3 * nc3) break;
        const int a = o / nc3, b = o - a * nc3, sa = a / n2, ia = a - sa * n2;
        const double2* p = P2 + ((long long)(X3 * 2 + sa) * n2 + ia) * K + l * n;
        double re = acc[q].x, im = acc[q].y;
        for (int c = 0; c < n; ++c) {
          const double2 u = p[c], t = T[(sa * n + c) * nc3 + b];
          re += u.x * t.x + u.y * t.y;   // conj(u) t
          im += u.x * t.y - u.y * t.x;
        }
        acc[q] = double2{re, im};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int o = threadIdx.x + 256 * q;
    if (o >= nc3 * nc3) break;
    const int a = o / nc3, b = o - a * nc3;
    D3[((long long)X3 * 9 + d3) * nc3 * nc3 + (long long)b * nc3 + a] = acc[q];
  }
}

// alpha[r] = <ar, r> / <ar, ar> for the minimal-residual smoother (FP64 dots; zero when ar = 0)
__global__ void k_mr_alpha(int nrhs, const double2* __restrict__ num, const double2* __restrict__ den,
                           double2* __restrict__ alpha) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double d = den[r].x;
  alpha[r] = d > 0.0 ? double2{num[r].x / d, num[r].y / d} : double2{0.0, 0.0};
}

}  // namespace

void launch_gs2(int Vc, int Vc3, int n, int n2, const int* slot_of, const double2* tv, double2* P2, int* bad,
                hipStream_t st) {
  k_gs2<<<2 * Vc3, 256, 0, st>>>(Vc, n, n2, slot_of, tv, P2, bad);
}

void launch_restrict2(dd_dtype vt, int Vc, int Vc3, int n, int n2, const int* slot_of, const void* P2, int nrhs,
                      const void* v, void* out, hipStream_t st) {
  const dim3 grid(Vc3, nrhs);
  const double bytes = (double)nrhs * Vc * 2 * n * vector_pair_bytes(vt) + (double)Vc * 2 * n * n2 * vector_pair_bytes(vt);
  const double flops = 8.0 * nrhs * Vc * 2 * n * n2;
  if (vt == DD_F64)
    DD_TIMED("k_restrict2", st, bytes, flops,
             (k_restrict2<double2, double2><<<grid, 256, 0, st>>>(Vc, Vc3, n, n2, slot_of, (const double2*)P2,
                                                                  (const double2*)v, (double2*)out)));
  else
    DD_TIMED("k_restrict2", st, bytes, flops,
             (k_restrict2<float2, float2><<<grid, 256, 0, st>>>(Vc, Vc3, n, n2, slot_of, (const float2*)P2,
                                                                (const float2*)v, (float2*)out)));
}

void launch_prolong2(dd_dtype vt, int Vc, int Vc3, int n, int n2, const int* l3_of, const int* loc_of, const void* P2,
                     int nrhs, const void* y, void* out, hipStream_t st) {
  const long long tot = (long long)Vc * 2 * n;
  const unsigned nb = (unsigned)((tot + 255) / 256);
  const double bytes = (double)nrhs * Vc * 2 * n * vector_pair_bytes(vt) + (double)Vc * 2 * n * n2 * vector_pair_bytes(vt);
  const double flops = 8.0 * nrhs * Vc * 2 * n * n2;
  if (vt == DD_F64)
    DD_TIMED("k_prolong2", st, bytes, flops,
             (k_prolong2<double2, double2><<<nb, 256, 0, st>>>(Vc, Vc3, n, n2, l3_of, loc_of, (const double2*)P2,
                                                               (const double2*)y, (double2*)out, nrhs)));
  else
    DD_TIMED("k_prolong2", st, bytes, flops,
             (k_prolong2<float2, float2><<<nb, 256, 0, st>>>(Vc, Vc3, n, n2, l3_of, loc_of, (const float2*)P2,
                                                             (const float2*)y, (float2*)out, nrhs)));
}

void launch_galerkin3(const GeomDev& g2, int Vc3, int n, int n2, const int* slot_of, const int* l3_of,
                      const int* loc_of, const double2* Dc64, const double2* P2, double2* D3, hipStream_t st) {
  const size_t shm = sizeof(double2) * (size_t)2 * n * 2 * n2;
  k_galerkin3<<<9 * Vc3, 256, shm, st>>>(g2, n, n2, slot_of, l3_of, loc_of, Dc64, P2, D3);
}

void launch_mr_alpha(int nrhs, const double2* num, const double2* den, double2* alpha, hipStream_t st) {
  k_mr_alpha<<<(nrhs + 63) / 64, 64, 0, st>>>(nrhs, num, den, alpha);
}

// Packed layouts: canonical <-> packed fine vectors, link re-layout and
// storage-dtype conversions.
#include "dd_internal.h"

namespace {

// one thread per (packed site, rhs): canonical [rhs][lex][12] <-> packed [rhs][12][V]
template <typename Tv, typename R>
__global__ void k_pack_fine(GeomDev g, int nrhs, const double2* __restrict__ canon, Tv* __restrict__ packed) {
  long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (I >= g.V) return;
  SiteLoc s = decode_site(g, I);
  long long x = lex_site(g, s);
  const double2* src = canon + ((long long)r * g.V + x) * 12;
  Tv* dst = packed + (long long)r * 12 * g.V + I;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    double2 v = src[c];
    st<Tv, double>(dst + c * g.V, cx<double>{v.x, v.y});
  }
}

template <typename Tv, typename R>
__global__ void k_unpack_fine(GeomDev g, int nrhs, const Tv* __restrict__ packed, double2* __restrict__ canon) {
  long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (I >= g.V) return;
  SiteLoc s = decode_site(g, I);
  long long x = lex_site(g, s);
  double2* dst = canon + ((long long)r * g.V + x) * 12;
  const Tv* src = packed + (long long)r * 12 * g.V + I;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cx<double> v = ld<double, Tv>(src + c * g.V);
    dst[c] = make_double2(v.re, v.im);
  }
}

// canonical links [lex][4][3][3] -> packed [mu][9][V] (FP64)
__global__ void k_pack_links(GeomDev g, const double2* __restrict__ canon, double2* __restrict__ links) {
  long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= g.V) return;
  SiteLoc s = decode_site(g, I);
  long long x = lex_site(g, s);
  const double2* src = canon + x * 36;
#pragma unroll
  for (int k = 0; k < 36; ++k) links[k * g.V + I] = src[k];
}

// Storage conversions, round to nearest even.  FP16 and BF16 copies are made
// from the FP32 copy (FP64 -> FP32 -> FP16/BF16): two separate roundings, so
// the compiler cannot merge them into one FP64 -> FP16 rounding.
__global__ void k_to_f32(const double2* __restrict__ s, float2* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = make_float2((float)s[i].x, (float)s[i].y);
}
__global__ void k_f32_to_f16(const float2* __restrict__ s, __half2* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = __floats2half2_rn(s[i].x, s[i].y);
}
__global__ void k_f32_to_bf16(const float2* __restrict__ s, bf16x2* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    uint32_t lo = f32_to_bf16_bits(s[i].x);
    uint32_t hi = f32_to_bf16_bits(s[i].y);
    d[i].u = lo | (hi << 16);
  }
}
__global__ void k_copy2(const double2* __restrict__ s, double2* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ void k_vec_f64_to_f32(const double2* __restrict__ s, float2* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = make_float2((float)s[i].x, (float)s[i].y);
}
__global__ void k_vec_f32_to_f64(const float2* __restrict__ s, double2* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = make_double2((double)s[i].x, (double)s[i].y);
}

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_pack_fine(const GeomDev& g, dd_dtype vt, int nrhs, const double2* canon, void* packed,
                      hipStream_t st) {
  dim3 grid(nblocks(g.V, 256), nrhs);
  if (vt == DD_F64)
    k_pack_fine<double2, double><<<grid, 256, 0, st>>>(g, nrhs, canon, (double2*)packed);
  else
    k_pack_fine<float2, float><<<grid, 256, 0, st>>>(g, nrhs, canon, (float2*)packed);
}

void launch_unpack_fine(const GeomDev& g, dd_dtype vt, int nrhs, const void* packed, double2* canon,
                        hipStream_t st) {
  dim3 grid(nblocks(g.V, 256), nrhs);
  if (vt == DD_F64)
    k_unpack_fine<double2, double><<<grid, 256, 0, st>>>(g, nrhs, (const double2*)packed, canon);
  else
    k_unpack_fine<float2, float><<<grid, 256, 0, st>>>(g, nrhs, (const float2*)packed, canon);
}

void launch_pack_links(const GeomDev& g, const double2* canon, double2* links64, hipStream_t st) {
  k_pack_links<<<nblocks(g.V, 256), 256, 0, st>>>(g, canon, links64);
}

void launch_convert_pairs(dd_dtype to, const double2* src64, const float2* src32, void* dst, long long n,
                          hipStream_t st) {
  unsigned nb = nblocks(n, 256);
  switch (to) {
    case DD_F64: k_copy2<<<nb, 256, 0, st>>>(src64, (double2*)dst, n); break;
    case DD_F32: k_to_f32<<<nb, 256, 0, st>>>(src64, (float2*)dst, n); break;
    case DD_F16: k_f32_to_f16<<<nb, 256, 0, st>>>(src32, (__half2*)dst, n); break;
    case DD_BF16: k_f32_to_bf16<<<nb, 256, 0, st>>>(src32, (bf16x2*)dst, n); break;
  }
}

void launch_vec_convert(dd_dtype from, dd_dtype to, const void* src, void* dst, long long n, hipStream_t st) {
  unsigned nb = nblocks(n, 256);
  if (from == DD_F64 && to != DD_F64)
    k_vec_f64_to_f32<<<nb, 256, 0, st>>>((const double2*)src, (float2*)dst, n);
  else if (from != DD_F64 && to == DD_F64)
    k_vec_f32_to_f64<<<nb, 256, 0, st>>>((const float2*)src, (double2*)dst, n);
  else if (from == DD_F64)
    k_copy2<<<nb, 256, 0, st>>>((const double2*)src, (double2*)dst, n);
  else
    hipMemcpyAsync(dst, src, n * sizeof(float2), hipMemcpyDeviceToDevice, st);
}

// ---------------------------------------------------------------------------
// Random starting vectors: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// keyed by the seed, counter = entry index, and the Box-Muller transform
// (one 4x32 draw per complex entry: two uniforms -> real and imaginary part).
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
  uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__global__ void k_gauss(unsigned long long seed, long long n, double2* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
  double u1 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
  double u2 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
  double rr = sqrt(-2.0 * log(u1));
  double s, co;
  sincospi(2.0 * u2, &s, &co);
  out[i] = make_double2(rr * co, rr * s);
}

}  // namespace

void launch_gauss(unsigned long long seed, long long n, double2* out, hipStream_t st) {
  k_gauss<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(seed, n, out);
}

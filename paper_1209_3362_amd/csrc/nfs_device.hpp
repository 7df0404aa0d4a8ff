// Device helpers shared by the library's HIP kernels: complex arithmetic,
// in-register DFTs with compile-time twiddles, exact integer square roots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace nfs {
namespace dev {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
// a * w
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}

// ---------------------------------------------------------------------------
// Raw buffer stores: a buffer resource covers `bytes` bytes from its base;
// the hardware drops a store whose byte offset lies at or past that range,
// so kDropOffset marks an element that is not written, without a branch.
using BufferRsrc = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kDropOffset = 0x80000000u;
// Word 3 of a gfx9 buffer descriptor: 32-bit data format, no swizzle.
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ BufferRsrc make_buffer(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, static_cast<short>(0), static_cast<int>(bytes),
                                           kBufferWord3);
}
__device__ __forceinline__ void buffer_store_u32(uint32_t v, BufferRsrc r, uint32_t byte_offset) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, static_cast<int>(byte_offset), 0, 0);
}

// Storage types of the resident spectra (values of nfs_desc.spec_dtype).
constexpr int kSpecF32 = 0, kSpecBF16 = 1, kSpecF16 = 2;

// (re, im) rounded to BF16 / FP16 (nearest, ties to even), re in the low
// half of the word.
__device__ __forceinline__ uint32_t pack_bf16(float2 v) {
  const __bf16 a = static_cast<__bf16>(v.x), b = static_cast<__bf16>(v.y);
  return uint32_t(__builtin_bit_cast(uint16_t, a)) |
         (uint32_t(__builtin_bit_cast(uint16_t, b)) << 16);
}
__device__ __forceinline__ uint32_t pack_f16(float2 v) {
  const _Float16 a = static_cast<_Float16>(v.x), b = static_cast<_Float16>(v.y);
  return uint32_t(__builtin_bit_cast(uint16_t, a)) |
         (uint32_t(__builtin_bit_cast(uint16_t, b)) << 16);
}
// Inverses (exact).
__device__ __forceinline__ float2 unpack_bf16(uint32_t w) {
  return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}
__device__ __forceinline__ float2 unpack_f16(uint32_t w) {
  return make_float2(static_cast<float>(__builtin_bit_cast(_Float16, uint16_t(w & 0xffffu))),
                     static_cast<float>(__builtin_bit_cast(_Float16, uint16_t(w >> 16))));
}

// Largest e with bound * 2^e <= 65504 (the FP16 maximum), 0 for a bound
// that is not positive and finite, clamped to [-100, 100].
__device__ __forceinline__ int f16_exponent(double bound) {
  if (!(bound > 0.0) || !isfinite(bound)) return 0;
  int k = 0;
  (void)frexp(65504.0 / bound, &k);
  int e = k - 1;
  while (e > -100 && ldexp(bound, e) > 65504.0) --e;
  while (e < 100 && ldexp(bound, e + 1) <= 65504.0) ++e;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

__device__ __forceinline__ void buffer_store(float2 v, BufferRsrc r, uint32_t byte_offset) {
  using U2 = __attribute__((ext_vector_type(2))) unsigned;
  U2 bits;
  bits.x = __float_as_uint(v.x);
  bits.y = __float_as_uint(v.y);
  __builtin_amdgcn_raw_buffer_store_b64(bits, r, static_cast<int>(byte_offset), 0, 0);
}

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2*pi*j/n, evaluated in double: the angle is split
// into its octant and a remainder in [0, pi/4], where Taylor series converge
// to double precision in 14 terms; results are exact at multiples of pi/2.
struct CosSin {
  double c, s;
};

constexpr double kPiD = 3.14159265358979323846264338327950288;

constexpr double series_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double series_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

constexpr CosSin cos_sin_2pi(long j, long n) {
  j %= n;
  if (j < 0) j += n;
  const long o = (8 * j) / n;       // octant
  const long r = 8 * j - o * n;     // remainder, angle = pi/4 * (o + r/n)
  const double f = double(r) / double(n);
  double ca = 0, sa = 0;            // cos/sin of the angle within its quadrant
  if ((o & 1) == 0) {
    const double a = 0.25 * kPiD * f;
    ca = (r == 0) ? 1.0 : series_cos(a);
    sa = (r == 0) ? 0.0 : series_sin(a);
  } else {
    const double b = 0.25 * kPiD * (1.0 - f);  // pi/2 - angle in quadrant
    ca = series_sin(b);
    sa = series_cos(b);
  }
  const long q = o >> 1;
  if (q == 0) return CosSin{ca, sa};
  if (q == 1) return CosSin{-sa, ca};
  if (q == 2) return CosSin{-ca, -sa};
  return CosSin{sa, -ca};
}

// W_N^J = exp(-2 pi i J / N), rounded once to float.
template <int N, int J>
struct Twiddle {
  static constexpr CosSin v = cos_sin_2pi(J, N);
  static constexpr float re = float(v.c);
  static constexpr float im = float(-v.s);
};

// d * W_N^J with the trivial factors done without multiplications.
template <int N, int J>
__device__ __forceinline__ float2 twiddle_mul(float2 d) {
  constexpr float kR = 0.70710678118654752440f;
  if constexpr (J == 0) {
    return d;
  } else if constexpr (4 * J == N) {            // -i
    return make_float2(d.y, -d.x);
  } else if constexpr (8 * J == N) {            // (1 - i)/sqrt(2)
    return make_float2(kR * (d.x + d.y), kR * (d.y - d.x));
  } else if constexpr (8 * J == 3 * N) {        // (-1 - i)/sqrt(2)
    return make_float2(kR * (d.y - d.x), -kR * (d.x + d.y));
  } else {
    return cmul(d, make_float2(Twiddle<N, J>::re, Twiddle<N, J>::im));
  }
}

// ---------------------------------------------------------------------------
// Compile-time loops.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

template <int P>
constexpr int bitrev(int k) {
  int r = 0;
  for (int b = 0; b < ilog2(P); ++b) r |= ((k >> b) & 1) << (ilog2(P) - 1 - b);
  return r;
}

// ---------------------------------------------------------------------------
// In-register radix-2 decimation-in-frequency DFT of P points:
// X[k] = sum_j v[j] W_P^{jk}. On return X[k] sits in v[bitrev<P>(k)].
template <int P, int S, int J>
__device__ __forceinline__ void dif_pair(float2 (&v)[P]) {
#pragma unroll
  for (int b = 0; b < P; b += 2 * S) {
    const float2 a = v[b + J], c = v[b + J + S];
    v[b + J] = cadd(a, c);
    v[b + J + S] = twiddle_mul<2 * S, J>(csub(a, c));
  }
}

template <int P, int S, int... J>
__device__ __forceinline__ void dif_stage(float2 (&v)[P], std::integer_sequence<int, J...>) {
  (dif_pair<P, S, J>(v), ...);
}

template <int P, int S>
__device__ __forceinline__ void dif_stages(float2 (&v)[P]) {
  dif_stage<P, S>(v, std::make_integer_sequence<int, S>{});
  if constexpr (S > 1) dif_stages<P, S / 2>(v);
}

template <int P>
__device__ __forceinline__ void dft(float2 (&v)[P]) {
  if constexpr (P > 1) dif_stages<P, P / 2>(v);
}

// ---------------------------------------------------------------------------
// Exact integer square roots.
__device__ __forceinline__ uint64_t isqrt_dev(uint64_t v) {
  uint64_t s = uint64_t(sqrt(double(v)));
  while (s > 0 && s * s > v) --s;
  while ((s + 1) * (s + 1) <= v) ++s;
  return s;
}
// Smallest s >= 0 with s*s >= v.
__device__ __forceinline__ int64_t ceil_sqrt_dev(int64_t v) {
  if (v <= 0) return 0;
  const int64_t s = int64_t(isqrt_dev(uint64_t(v)));
  return s * s == v ? s : s + 1;
}

// Bin of mode (ky, kx): isqrt(|k|^2 nb^2) / (n/2), or -1 outside every bin.
__device__ __forceinline__ int bin_of_dev(int n, int nb, int ky, int kx) {
  const uint64_t r2 = uint64_t(int64_t(kx) * kx + int64_t(ky) * ky);
  const uint64_t b = isqrt_dev(r2 * uint64_t(nb) * uint64_t(nb)) / uint64_t(n / 2);
  return b < uint64_t(nb) ? int(b) : -1;
}

// Slot layout of a stored spectrum: the columns k_x are cut into tiles of
// 8; tile t keeps the transform-order rows r with |k_y(r)| <= R_t (every row
// holding a stored mode of the tile) as consecutive runs of 8 slots, rows in
// the order 0..R_t, n - R_t..n - 1, from slot base_t, so a column-pass
// workgroup writes one contiguous block. tiles = {base_0 .. base_T,
// R_0 .. R_{T-1}}, T = n / 16. Slots of rows kept but of modes that are not
// stored (|k| >= n/2) hold the transform's values and are never binned.
// Returns the slot of (r, kx), or -1 when row r is not kept in kx's tile.
__device__ __forceinline__ int ring_slot(int n, const int32_t* __restrict__ tiles, int r,
                                         int kx) {
  const int t = kx >> 3;
  const int R = tiles[(n >> 4) + 1 + t];
  // R = n/2 marks a tile that keeps all n rows (full half-plane plans).
  if (R >= (n >> 1)) return tiles[t] + r * 8 + (kx & 7);
  const int ky = r < (n >> 1) ? r : r - n;
  if (ky > R || -ky > R) return -1;
  const int rank = r <= R ? r : r - (n - 2 * R - 1);
  return tiles[t] + rank * 8 + (kx & 7);
}

// Ring b = modes with lo <= |k|^2 < hi (same rule as bin_of_dev).
__device__ __forceinline__ void ring_bounds_dev(int n, int nb, int b, int64_t* lo,
                                                int64_t* hi) {
  const int64_t m = n / 2, q = int64_t(nb) * nb;
  const int64_t a = int64_t(b) * m, c = int64_t(b + 1) * m;
  *lo = (a * a + q - 1) / q;
  *hi = (c * c + q - 1) / q;
}

}  // namespace dev
}  // namespace nfs

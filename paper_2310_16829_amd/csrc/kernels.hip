// gfx950 kernels of the LMA hot path.
//
// One multislice step (Fig. multislice_pseudocode) is two passes over the batch of waves:
//   row pass    : row IFFT (finishes the previous step's inverse transform), transmission
//                 exp(i sigma v_j), row FFT
//   column pass : column FFT, Fresnel propagator with band limit, column IFFT
// Between passes a wave lives in HBM in the mixed domain (x transformed, y spatial), so each
// step reads and writes every pixel twice: 32 bytes per pixel per slice per wave.
//
// Transforms are Stockham FFTs: lengths 2^a run radix 8 (then 4 or 2) with E = 8 elements
// per thread, lengths 3 * 2^a and 5 * 2^a run the odd radix first, then radix 4 (then 2), with
// E = 12 or 20. N/E threads per transform each hold elements j + (N/E) m for m < E before
// every stage and after the last one, so consecutive transforms need no exchange; stages in
// between exchange through LDS. Twiddles come from FP64-computed tables rounded to FP32.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <atomic>

#include "kernels.hpp"

namespace lma {
namespace dev {

// ------------------------------------------------------------------------------------------
// complex helpers
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// DIR = -1: forward transform (kernel exp(-2 pi i ...)), DIR = +1: inverse
template <int DIR>
__device__ __forceinline__ float2 mul_unit_i(float2 a) {  // a * (DIR * i)
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
template <int DIR>
__device__ __forceinline__ float2 conj_if_inv(float2 w) { return DIR < 0 ? w : make_float2(w.x, -w.y); }

template <int DIR>
__device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}
template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_unit_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}
template <int DIR>
__device__ __forceinline__ void dft8(float2* a) {
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  const float r = 0.70710678118654752440f;
  // o1 *= W8^1, o2 *= W8^2, o3 *= W8^3 (W8 = exp(DIR * 2 pi i / 8))
  if (DIR < 0) {
    o1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
    o3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  } else {
    o1 = make_float2(r * (o1.x - o1.y), r * (o1.x + o1.y));
    o3 = make_float2(-r * (o3.x + o3.y), r * (o3.x - o3.y));
  }
  o2 = mul_unit_i<DIR>(o2);
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// 3-point DFT: X0 = a0 + (a1 + a2), X1,2 = a0 - (a1 + a2)/2 +- DIR i sin(2 pi/3) (a1 - a2)
template <int DIR>
__device__ __forceinline__ void dft3(float2* a) {
  const float s3 = 0.86602540378443864676f;   // sin(2 pi / 3)
  const float2 t1 = cadd(a[1], a[2]);
  const float2 t2 = make_float2(a[0].x - 0.5f * t1.x, a[0].y - 0.5f * t1.y);
  const float2 d = mul_unit_i<DIR>(csub(a[1], a[2]));
  a[0] = cadd(a[0], t1);
  a[1] = make_float2(t2.x + s3 * d.x, t2.y + s3 * d.y);
  a[2] = make_float2(t2.x - s3 * d.x, t2.y - s3 * d.y);
}
// 5-point DFT from the symmetric sums t1 = a1 + a4, t2 = a2 + a3 and differences
// t3 = a1 - a4, t4 = a2 - a3 (w = exp(DIR 2 pi i / 5); c_k, s_k = cos, sin of 2 pi k / 5):
//   X1,4 = a0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4)
//   X2,3 = a0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4)
template <int DIR>
__device__ __forceinline__ void dft5(float2* a) {
  const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
  const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
  const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
  const float2 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
  const float2 r1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
  const float2 r2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
  const float2 i1 = mul_unit_i<DIR>(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const float2 i2 = mul_unit_i<DIR>(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  a[0] = cadd(a[0], cadd(t1, t2));
  a[1] = cadd(r1, i1);
  a[4] = csub(r1, i1);
  a[2] = cadd(r2, i2);
  a[3] = csub(r2, i2);
}

// c + w b with four FMAs, and 2 b - s with two: a twiddled butterfly pair a +- w b becomes
// s = a + w b and d = 2 a - s, six operations instead of eight
__device__ __forceinline__ float2 cfma(float2 b, float2 w, float2 c) {
  return make_float2(__builtin_fmaf(b.x, w.x, __builtin_fmaf(-b.y, w.y, c.x)),
                     __builtin_fmaf(b.x, w.y, __builtin_fmaf(b.y, w.x, c.y)));
}
__device__ __forceinline__ float2 ctwice_minus(float2 b, float2 s) {
  return make_float2(__builtin_fmaf(2.f, b.x, -s.x), __builtin_fmaf(2.f, b.y, -s.y));
}

// 8-point DFT with optional input twiddles w[m - 1] (m = 1..7, already conjugated for the
// direction) folded into its first butterfly level. Z34: inputs 3 and 4 are known zeros (not
// read); SKIP34: outputs 3 and 4 are not needed (not computed). Levels: pairs (0,4), (2,6),
// (1,5), (3,7); then the two 4-point combinations; then the W8 twiddles and the final pairs.
#ifndef LMA_FUSED_TW
#define LMA_FUSED_TW 1
#endif
template <int DIR, bool TW, bool Z34, bool SKIP34>
__device__ __forceinline__ void dft8x(float2* a, const float2* w) {
  static_assert(!(TW && Z34), "known-zero inputs only without twiddles (the first stage)");
  float2 s04, d04, s26, d26, s15, d15, s37, d37;
  if constexpr (TW && !LMA_FUSED_TW) {
    const float2 a1 = cmul(a[1], w[0]), a2 = cmul(a[2], w[1]), a3 = cmul(a[3], w[2]), a4 = cmul(a[4], w[3]);
    const float2 a5 = cmul(a[5], w[4]), a6 = cmul(a[6], w[5]), a7 = cmul(a[7], w[6]);
    s04 = cadd(a[0], a4);
    d04 = csub(a[0], a4);
    s26 = cadd(a2, a6);
    d26 = csub(a2, a6);
    s15 = cadd(a1, a5);
    d15 = csub(a1, a5);
    s37 = cadd(a3, a7);
    d37 = csub(a3, a7);
  } else if constexpr (TW) {
    s04 = cfma(a[4], w[3], a[0]);
    d04 = ctwice_minus(a[0], s04);
    const float2 b2 = cmul(a[2], w[1]);
    s26 = cfma(a[6], w[5], b2);
    d26 = ctwice_minus(b2, s26);
    const float2 b1 = cmul(a[1], w[0]);
    s15 = cfma(a[5], w[4], b1);
    d15 = ctwice_minus(b1, s15);
    const float2 b3 = cmul(a[3], w[2]);
    s37 = cfma(a[7], w[6], b3);
    d37 = ctwice_minus(b3, s37);
  } else if constexpr (Z34) {
    s04 = a[0];
    d04 = a[0];
    s26 = cadd(a[2], a[6]);
    d26 = csub(a[2], a[6]);
    s15 = cadd(a[1], a[5]);
    d15 = csub(a[1], a[5]);
    s37 = a[7];
    d37 = make_float2(-a[7].x, -a[7].y);
  } else {
    s04 = cadd(a[0], a[4]);
    d04 = csub(a[0], a[4]);
    s26 = cadd(a[2], a[6]);
    d26 = csub(a[2], a[6]);
    s15 = cadd(a[1], a[5]);
    d15 = csub(a[1], a[5]);
    s37 = cadd(a[3], a[7]);
    d37 = csub(a[3], a[7]);
  }
  // the two 4-point DFTs (evens e, odds o)
  const float2 e0 = cadd(s04, s26), e2 = csub(s04, s26);
  const float2 i26 = mul_unit_i<DIR>(d26);
  const float2 e1 = cadd(d04, i26), e3 = csub(d04, i26);
  float2 o0 = cadd(s15, s37), o2 = csub(s15, s37);
  const float2 i37 = mul_unit_i<DIR>(d37);
  float2 o1 = cadd(d15, i37), o3 = csub(d15, i37);
  const float r = 0.70710678118654752440f;
  // o1 *= W8^1, o2 *= W8^2, o3 *= W8^3 (W8 = exp(DIR * 2 pi i / 8))
  if (DIR < 0) {
    o1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
    o3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  } else {
    o1 = make_float2(r * (o1.x - o1.y), r * (o1.x + o1.y));
    o3 = make_float2(-r * (o3.x + o3.y), r * (o3.x - o3.y));
  }
  o2 = mul_unit_i<DIR>(o2);
  a[0] = cadd(e0, o0);
  a[1] = cadd(e1, o1);
  a[2] = cadd(e2, o2);
  a[5] = csub(e1, o1);
  a[6] = csub(e2, o2);
  a[7] = csub(e3, o3);
  if constexpr (!SKIP34) {
    a[3] = cadd(e3, o3);
    a[4] = csub(e0, o0);
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dft_r(float2* a) {
  if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 5) dft5<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 3) dft3<DIR>(a);
  else if constexpr (R == 2) dft2<DIR>(a[0], a[1]);
}

// ------------------------------------------------------------------------------------------
// stage schedule. 2^a: radix 8 while possible, the remaining factor (2 or 4) last, E = 8
// (E = 16 at 1024 points, so that a line is one wavefront's: 8.8.8.2, exchanges without
// workgroup barriers; measured +17-23 % over two wavefronts per line).
// 3 * 2^a and 5 * 2^a: the odd radix, then radix 4, then a 2 if needed, E = 4 x the odd factor
// (every radix of the schedule divides E).
// ------------------------------------------------------------------------------------------
__host__ __device__ constexpr int fft_odd(int n) { while (n > 1 && n % 2 == 0) n /= 2; return n; }
__host__ __device__ constexpr bool fft_pow2(int n) { return fft_odd(n) == 1; }
__host__ __device__ constexpr int fft_elems(int n) { return fft_pow2(n) ? (n == 1024 ? 16 : 8) : 4 * fft_odd(n); }
__host__ __device__ constexpr int fft_log2(int n) { int a = 0; while (n > 1) { n /= 2; ++a; } return a; }
__host__ __device__ constexpr int fft_full8(int n) { int s = 0; while (n >= 8) { n /= 8; ++s; } return s; }
__host__ __device__ constexpr int fft_rest(int n) { while (n >= 8) n /= 8; return n; }
__host__ __device__ constexpr int fft_nstages(int n) {
  return fft_pow2(n) ? fft_full8(n) + (fft_rest(n) > 1 ? 1 : 0)
                     : 1 + fft_log2(n / fft_odd(n)) / 2 + fft_log2(n / fft_odd(n)) % 2;
}
__host__ __device__ constexpr int fft_radix_base(int n, int s) {
  if (fft_pow2(n)) return s < fft_full8(n) ? 8 : fft_rest(n);
  return s == 0 ? fft_odd(n) : (s <= fft_log2(n / fft_odd(n)) / 2 ? 4 : 2);
}
// Radix schedules: the same radices in another order (every order is a valid Stockham
// transform, the per-thread element count E is divisible by each). 0: the base order; 1: its
// last stage first; 2: its first stage last. Lengths whose radices are all equal have one.
__host__ __device__ constexpr int fft_radix(int n, int s, int sched = 0) {
  const int ns = fft_nstages(n);
  const int b = sched == 1 ? (s == 0 ? ns - 1 : s - 1) : sched == 2 ? (s == ns - 1 ? 0 : s + 1) : s;
  return fft_radix_base(n, b);
}
__host__ __device__ constexpr int fft_span(int n, int s, int sched = 0) {  // product of the radices before stage s
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fft_radix(n, i, sched);
  return p;
}
// b mod NS and b / NS for b >= 0 (masks and shifts when NS is a power of two)
template <int NS>
__device__ __forceinline__ int mod_c(int b) { return fft_pow2(NS) ? (b & (NS - 1)) : (int)((unsigned)b % (unsigned)NS); }
template <int NS>
__device__ __forceinline__ int div_c(int b) { return (int)((unsigned)b / (unsigned)NS); }
// transform lengths the passes are built for
__host__ __device__ constexpr bool fft_length_ok(int n) {
  return (fft_pow2(n) && n >= 16 && n <= 2048) || n == 96 || n == 192 || n == 384 || n == 640;
}

// ------------------------------------------------------------------------------------------
// twiddles: for every stage after the first, the factors w^m (m = 1..r-1) of each of the
// thread's E/r butterflies, from the FP64-derived table. Lengths 2^a and 3 * 2^a hold all of
// them in registers for the whole pass. Lengths 5 * 2^a (20 elements per thread) would need
// 55 registers pairs; they read w from the table at each stage (one load per butterfly) and
// form w^2, w^3 by complex products (FP32, a few ulp).
// ------------------------------------------------------------------------------------------
__host__ __device__ constexpr bool tw_in_regs(int n) { return fft_odd(n) != 5; }
__host__ __device__ constexpr int tw_off(int n, int s, int sched = 0) {
  int o = 0;
  for (int i = 1; i < s; ++i) o += fft_elems(n) - fft_elems(n) / fft_radix(n, i, sched);
  return o;
}
__host__ __device__ constexpr int tw_count(int n, int sched = 0) {
  return tw_in_regs(n) && tw_off(n, fft_nstages(n), sched) > 0 ? tw_off(n, fft_nstages(n), sched) : 1;
}

template <int N, int S, int SCHED = 0>
__device__ __forceinline__ void tw_load_stage(float2* w, const float2* __restrict__ tab, int j) {
  constexpr int E = fft_elems(N);
  constexpr int r = fft_radix(N, S, SCHED), Ns = fft_span(N, S, SCHED), Q = E / r, T = N / E;
  constexpr int off = tw_off(N, S, SCHED);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = mod_c<Ns>(j + T * q);
#pragma unroll
    for (int m = 1; m < r; ++m) w[off + q * (r - 1) + (m - 1)] = tab[m * k * (N / (Ns * r))];
  }
}

template <int N, int SCHED = 0>
__device__ __forceinline__ void tw_load(float2* w, const float2* __restrict__ tab, int j) {
  constexpr int ns = fft_nstages(N);
  if constexpr (!tw_in_regs(N)) return;
  if constexpr (ns > 1) tw_load_stage<N, 1, SCHED>(w, tab, j);
  if constexpr (ns > 2) tw_load_stage<N, (ns > 2 ? 2 : 1), SCHED>(w, tab, j);
  if constexpr (ns > 3) tw_load_stage<N, (ns > 3 ? 3 : 1), SCHED>(w, tab, j);
  if constexpr (ns > 4) tw_load_stage<N, (ns > 4 ? 4 : 1), SCHED>(w, tab, j);
  if constexpr (ns > 5) tw_load_stage<N, (ns > 5 ? 5 : 1), SCHED>(w, tab, j);
}

// One transform's exchange slot inside the pass tile: position p lives at p + p/2^PAD (one
// pad element every 2^PAD keeps the stride-8 Stockham writes on distinct banks of the
// 64 x 4-byte LDS).
#ifndef LMA_SLOT_PAD
#define LMA_SLOT_PAD 3
#endif
#ifndef LMA_TILE_EXTRA_ROW
#define LMA_TILE_EXTRA_ROW 9
#endif
#ifndef LMA_TILE_EXTRA_COL
#define LMA_TILE_EXTRA_COL 3
#endif
__host__ __device__ constexpr int slot_pos(int p) { return p + (p >> LMA_SLOT_PAD); }
struct Slot {
  float2* base;
  __device__ __forceinline__ void put(int p, float2 v) const { base[slot_pos(p)] = v; }
  __device__ __forceinline__ float2 get(int p) const { return base[slot_pos(p)]; }
};

// Exchange ordering: a transform held by one wavefront only needs the compiler to keep its
// LDS writes before its reads (a wavefront's LDS operations execute in order); a transform
// spread over several wavefronts needs the workgroup barrier.
template <bool WAVE_LOCAL>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE_LOCAL) __builtin_amdgcn_wave_barrier();
  else __syncthreads();
}

// Pruning bits of a transform whose stages are all radix 8 with one butterfly per thread
// (E = 8): PRUNE_IN, its inputs at positions [3N/8, 5N/8) are zeros (the first stage's inputs
// 3 and 4); PRUNE_OUT, its outputs there are not needed (the last stage's outputs 3 and 4).
enum { PRUNE_IN = 1, PRUNE_OUT = 2 };
#ifndef LMA_PRUNE
#define LMA_PRUNE 1
#endif
#ifndef LMA_PRUNE_ROWS
#define LMA_PRUNE_ROWS 1
#endif
__host__ __device__ constexpr bool fft_prunable(int n) {
  if (!fft_pow2(n) || fft_elems(n) != 8) return false;
  for (int s = 0; s < fft_nstages(n); ++s)
    if (fft_radix(n, s) != 8) return false;
  return true;
}

template <int N, int DIR, int S, bool WL, int TAG = 0, int PRUNE = 0, int SCHED = 0>
__device__ __forceinline__ void fft_stage(float2 (&v)[fft_elems(N)], int j, const float2* w, const float2* twg,
                                          const Slot& slot) {
  constexpr int E = fft_elems(N);
  constexpr int r = fft_radix(N, S, SCHED);
  constexpr int Ns = fft_span(N, S, SCHED);
  constexpr int Q = E / r;
  constexpr int T = N / E;
  constexpr bool last = (S == fft_nstages(N) - 1);
  constexpr int off = tw_off(N, S, SCHED);
  static_assert(PRUNE == 0 || fft_prunable(N), "pruning needs radix-8 stages with E = 8");
  constexpr bool z34 = (PRUNE & PRUNE_IN) && S == 0;
  constexpr bool skip34 = (PRUNE & PRUNE_OUT) && last;
  if constexpr (r == 8 && tw_in_regs(N)) {
    // radix 8 with register twiddles: the twiddles folded into the first butterfly level
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      float2 a[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) a[m] = (z34 && (m == 3 || m == 4)) ? make_float2(0.f, 0.f) : v[q + m * Q];
      const int b = j + T * q;
      const int k = mod_c<Ns>(b);
      if constexpr (Ns > 1) {
        float2 tw7[7];
#pragma unroll
        for (int m = 1; m < 8; ++m) tw7[m - 1] = conj_if_inv<DIR>(w[off + q * 7 + (m - 1)]);
        dft8x<DIR, true, false, skip34>(a, tw7);
      } else {
        dft8x<DIR, false, z34, skip34>(a, nullptr);
      }
      if constexpr (last) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
          if (!(skip34 && (m == 3 || m == 4))) v[q + m * Q] = a[m];
      } else {
        const int base = div_c<Ns>(b) * Ns * 8 + k;
#pragma unroll
        for (int m = 0; m < 8; ++m) slot.put(base + m * Ns, a[m]);
      }
    }
    if constexpr (!last) {
      exchange_sync<WL>();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = slot.get(j + T * m);
      exchange_sync<WL>();
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 a[r];
#pragma unroll
    for (int m = 0; m < r; ++m) a[m] = v[q + m * Q];
    const int b = j + T * q;
    const int k = mod_c<Ns>(b);
    if constexpr (Ns > 1) {
      if constexpr (tw_in_regs(N)) {
#pragma unroll
        for (int m = 1; m < r; ++m) a[m] = cmul(a[m], conj_if_inv<DIR>(w[off + q * (r - 1) + (m - 1)]));
      } else {
        const float2 w1 = conj_if_inv<DIR>(twg[k * (N / (Ns * r))]);
        float2 wm = w1;
#pragma unroll
        for (int m = 1; m < r; ++m) {
          a[m] = cmul(a[m], wm);
          if (m + 1 < r) wm = cmul(wm, w1);
        }
      }
    }
    dft_r<r, DIR>(a);
    if constexpr (last) {
#pragma unroll
      for (int m = 0; m < r; ++m) v[q + m * Q] = a[m];
    } else {
      const int base = div_c<Ns>(b) * Ns * r + k;
#pragma unroll
      for (int m = 0; m < r; ++m) slot.put(base + m * Ns, a[m]);
    }
  }
  if constexpr (!last) {
    exchange_sync<WL>();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = slot.get(j + T * m);
    exchange_sync<WL>();
  }
}

// N-point transform of the E values held by thread j (of N/E); input and output at
// positions j + (N/E) m, natural order. w: the thread's register twiddles (tw_load); twg: the
// twiddle table (lengths whose twiddles are not held in registers). TAG gives a kernel its
// own instantiation: the embedding kernel sharing the passes' changed their register
// allocation (640 points: 33-58 spilled registers).
template <int N, int DIR, bool WL, int TAG = 0, int PRUNE = 0, int SCHED = 0>
__device__ __forceinline__ void fft(float2 (&v)[fft_elems(N)], int j, const float2* w, const float2* twg,
                                    const Slot& slot) {
  constexpr int ns = fft_nstages(N);
  static_assert(ns <= 6, "at most six stages");
  fft_stage<N, DIR, 0, WL, TAG, PRUNE, SCHED>(v, j, w, twg, slot);
  if constexpr (ns > 1) fft_stage<N, DIR, (ns > 1 ? 1 : 0), WL, TAG, PRUNE, SCHED>(v, j, w, twg, slot);
  if constexpr (ns > 2) fft_stage<N, DIR, (ns > 2 ? 2 : 0), WL, TAG, PRUNE, SCHED>(v, j, w, twg, slot);
  if constexpr (ns > 3) fft_stage<N, DIR, (ns > 3 ? 3 : 0), WL, TAG, PRUNE, SCHED>(v, j, w, twg, slot);
  if constexpr (ns > 4) fft_stage<N, DIR, (ns > 4 ? 4 : 0), WL, TAG, PRUNE, SCHED>(v, j, w, twg, slot);
  if constexpr (ns > 5) fft_stage<N, DIR, (ns > 5 ? 5 : 0), WL, TAG, PRUNE, SCHED>(v, j, w, twg, slot);
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
// logical blocks so that it touches one contiguous part of the shared tables.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  if (G & 7) return b;
  return (b & 7) * (G >> 3) + (b >> 3);
}

__device__ __forceinline__ int freq_index(int m, int n) { return m < (n + 1) / 2 ? m : m - n; }

// ------------------------------------------------------------------------------------------
// transmission t = exp(i sigma v), phase in FP64
// ------------------------------------------------------------------------------------------
__global__ void k_transmission(const float* __restrict__ v, float2* __restrict__ t, int64_t n, double sigma) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincos(sigma * (double)v[i], &s, &c);
  t[i] = make_float2((float)c, (float)s);
}

// ------------------------------------------------------------------------------------------
// slice pass
//
// Waves live in HBM in TW x TW tiles, in place for every pass: element (y, x) of wave w is at
//   w*XY + ((y/TW)*(nx/TW) + x/TW)*TW*TW + (y%TW)*TW + x%TW.
// A workgroup owns TW lines of one wave: a row pass (lines y, positions x) takes one tile row,
// a contiguous TW*nx block; a column pass (lines x, positions y) takes one tile column, ny/TW
// contiguous tiles. Lines are staged through an LDS tile (whole tiles move between HBM and LDS,
// with non-temporal hints), transformed with wavefront-local exchanges inside their LDS line,
// and written back to the same place. Between passes a wave is in the mixed domain (y
// spatial, x frequency). Tables read by column passes are stored transposed, [kx][ky].
// ------------------------------------------------------------------------------------------
enum { PASS_ROW = 0, PASS_COL = 1, PASS_INIT = 2, PASS_GATHER = 3, PASS_REDUCE = 4, PASS_ROW_WIN = 5, PASS_ROW_LAST = 6 };
// PASS_ROW_WIN / PASS_ROW_LAST: the row pass of waves propagated on windows of the cell
// (option (ii) of Sec. 4.2.1): each wave reads the cell's transmission at its own window;
// PASS_ROW_LAST stops after the transmission and leaves the window's wave in real space.
__host__ __device__ constexpr bool pass_rows(int mode) { return mode == PASS_ROW || mode == PASS_ROW_WIN || mode == PASS_ROW_LAST; }

// Wavefronts per workgroup for transforms that fit one wavefront (N <= 512): 8, one line each
// (8 prefetch registers pairs per thread instead of 16; 3-4 wavefronts per SIMD).
#ifndef LMA_WL_WAVES
#define LMA_WL_WAVES 8
#endif
#ifndef LMA_WL_WAVES_ROW
#define LMA_WL_WAVES_ROW 8
#endif
template <int N, int TW, int WLW = LMA_WL_WAVES, int KM = 2, int SCHED = 0>
struct PassCfg {
  static constexpr int E = fft_elems(N);                            // elements per thread
  static constexpr int T = N / E;                                   // threads per transform
  static constexpr bool WL = T <= 64;                               // transform inside one wavefront
  static constexpr int S = WL ? ((64 / T) < TW ? 64 / T : TW) : 1;  // transforms per wavefront
  static constexpr int WPT = WL ? 1 : T / 64;                       // wavefronts per transform
  // wavefronts per workgroup: single-wavefront transforms up to WLW lines at once; lines of
  // several wavefronts two at a time between the workgroup barriers (4 wavefronts at 1024
  // points, 8 at 2048)
  static constexpr int KMW = TW < KM ? TW : KM;   // multi-wavefront transforms in flight
  static constexpr int WAVES = WL ? ((TW / S) < WLW ? TW / S : WLW) : WPT * KMW;
  static constexpr int TPB = WAVES * S / WPT;                       // transforms in flight
  static constexpr int RPW = TW / TPB;                              // rounds per workgroup
  // LDS line stride: a padded slot plus a few elements, so that the TW lines touched by one
  // tile row fall on distinct banks (row passes stage a tile row by row, column passes
  // column by column: each has its own stride)
  static constexpr int RS_ROW = slot_pos(N - 1) + 1 + LMA_TILE_EXTRA_ROW;
  static constexpr int RS_COL = slot_pos(N - 1) + 1 + LMA_TILE_EXTRA_COL;
  static constexpr int NTW = tw_count(N, SCHED);
  static_assert(TPB >= 1 && TW % TPB == 0, "lines must split evenly over the workgroup");
};

struct PassArgs {
  float2* work;              // [B][tiles] waves, updated in place
  int nx, ny;
  int B;                     // waves in the batch
  const float2* table;       // ROW: t_j [ny][nx]; COL/GATHER/REDUCE: P^T [nx][ny]; INIT: spectrum^T
  const float2* tw;          // twiddles exp(-2 pi i t / N), t < N, N = line length
  const int64_t* wave_u;     // INIT: [B][2] lattice units of each wave's position
  int64_t Qx, Qy;
  void* basis;               // GATHER
  int D;
  const int32_t* comp;       // GATHER: detector pixel index [nx][ny] or -1
  const int32_t* wave_row;   // GATHER: basis row per wave; REDUCE: image index per wave
  int split_bf16;
  const uint32_t* mask;      // REDUCE: ring bits [nx][ny]
  double* img;
  int ndet;
  int64_t img_stride;
  double scale;
  int tnx, tny;              // ROW_WIN / ROW_LAST: the cell (table [tny][tnx]); window origin
  int hx, hy;                //   of wave w: its position in pixels minus (hx, hy)
  int zlo, zhi;              // tile columns [zlo, zhi) stay zero between passes (kx band gap);
                             //   INIT: the tile columns of the input spectrum's gap
  int zread;                 // row passes: skip reading tile columns [rlo, rhi), which hold
  int rlo, rhi;              //   zeros
  int prune;                 // column-type passes of 512- and 64-point lines (radix-8 stages, 8
                             //   per thread): the propagator vanishes at ky positions [3N/8, 5N/8)
                             //   of every column, so the column FFT does not form them and the
                             //   inverse FFT takes them as zeros
  // ROW over the waves of several specimens: wave w multiplies by the transmission of its own
  // specimen, spec_table[wave_spec[w]] + slice_off (null wave_spec: `table` for every wave)
  const float2* const* spec_table;
  const int32_t* wave_spec;
  int64_t slice_off;
};

__device__ __forceinline__ void split_bf16(float x, __hip_bfloat16& hi, __hip_bfloat16& lo) {
  hi = __float2bfloat16(x);
  lo = __float2bfloat16(x - __bfloat162float(hi));
}

__device__ __forceinline__ float2 load_stream(const float2* p) {
  const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
  return __builtin_bit_cast(float2, u);
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
  __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), reinterpret_cast<unsigned long long*>(p));
}
// A workgroup's HBM traffic comes in bursts (the next item's loads, the finished item's
// stores) between long stretches of FFT arithmetic; its wavefronts issue those bursts at a
// raised priority so that the memory pipeline is fed while the other workgroups on the CU
// compute (measured: +5 % on both passes at 512 points).
#ifndef LMA_PASS_PRIORITY
#define LMA_PASS_PRIORITY 2
#endif
// Passes address their items through buffer resources (32-bit offsets, 37 fewer registers per
// thread at 512 points for column items); elements in a gap are read and written at an offset
// past the item's extent, which reads zero and drops the store without touching memory, so the
// item's loads and stores carry no branches.
#ifndef LMA_BUFFER_IO_COL
#define LMA_BUFFER_IO_COL 1
#endif
#ifndef LMA_BUFFER_IO_ROW
#define LMA_BUFFER_IO_ROW 1
#endif
// Raw buffer access to one work item: the resource (base, byte extent) lives in scalar
// registers, each lane supplies a 32-bit byte offset; accesses past the extent read zero and
// drop stores.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t item_rsrc(const float2* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), 0, (int)bytes, 0x00020000);
}
constexpr int kOutOfItem = 0x0FFFFFFF;   // element offset beyond every item's extent
__device__ __forceinline__ float2 load_item_elem(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off * 8, 0, 2));
}
__device__ __forceinline__ void store_item_elem(__amdgpu_buffer_rsrc_t r, int off, float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off * 8, 0, 2);
}
// the same with the offset split into a per-lane part (voff) and a wavefront-uniform part
// (soff, bytes); the range check covers the per-lane part, so an empty extent still drops them
__device__ __forceinline__ float2 load_item_elem2(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
}
__device__ __forceinline__ void store_item_elem2(__amdgpu_buffer_rsrc_t r, int voff, int soff, float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 2);
}

__device__ __forceinline__ void memory_phase_begin() {
  if constexpr (LMA_PASS_PRIORITY > 0) __builtin_amdgcn_s_setprio(LMA_PASS_PRIORITY);
}
__device__ __forceinline__ void memory_phase_end() {
  if constexpr (LMA_PASS_PRIORITY > 0) __builtin_amdgcn_s_setprio(0);
}

// Element c of a work item (TW lines x N positions) <-> its LDS index and its offset from the
// item's first element in HBM. A row item (tile row g) is one contiguous block; a column item
// (tile column g) is N/TW tiles, one every nx/TW tiles.
template <int N, int TW, bool ROWS>
struct TileMap {
  static constexpr int TT = TW * TW;
  static constexpr int RS = ROWS ? PassCfg<N, TW>::RS_ROW : PassCfg<N, TW>::RS_COL;  // any wavefront count
  __device__ __forceinline__ static int64_t item_base(int g, int nx) {
    return ROWS ? (int64_t)g * TW * nx : (int64_t)g * TT;
  }
  __device__ __forceinline__ static void at(int c, int stride_q, int& lds, int& off) {
    const int q = c / TT, rem = c % TT;
    int line, pos;
    if constexpr (ROWS) {
      line = rem / TW;
      pos = q * TW + rem % TW;
      off = c;
    } else {
      line = rem % TW;
      pos = q * TW + rem / TW;
      off = q * stride_q + rem;
    }
    lds = line * RS + slot_pos(pos);
  }
};

// Work items of a pass are (line group g, wave w) pairs, item l = g*B + w. Workgroups are
// persistent: each walks a strided sequence of items, and the items of one XCD form one
// contiguous range (so an XCD reads one part of the shared tables).
struct ItemWalk {
  int l, end, step;
  __device__ __forceinline__ ItemWalk(int W) {
    const int G = gridDim.x, b = blockIdx.x;
    if ((G & 7) == 0 && (W & 7) == 0 && G >= 8) {
      const int x = b & 7, per = W >> 3;
      l = x * per + (b >> 3);
      end = (x + 1) * per;
      step = G >> 3;
    } else {
      l = b;
      end = W;
      step = G;
    }
  }
  __device__ __forceinline__ bool valid(int i) const { return i < end; }
};

// elements a thread stages per step when the item is not prefetched: the largest divisor of
// the per-thread count up to 16
constexpr int stage_chunk(int ept) {
  for (int c = 16; c > 1; --c)
    if (ept % c == 0) return c;
  return 1;
}

template <int MODE>
constexpr int pass_waves() { return pass_rows(MODE) ? LMA_WL_WAVES_ROW : LMA_WL_WAVES; }
// lines spanning several wavefronts in flight per workgroup: 2048-point lines one at a time
// (4-wavefront workgroups, two per CU: each exchange barrier holds one line's wavefronts; 13-15 %
// faster row, column and gather passes than two lines per 8-wavefront workgroup), except the
// initial waves (35 % slower so)
#ifndef LMA_KMW_2048
#define LMA_KMW_2048 1
#endif
template <int N, int MODE>
constexpr int pass_kmw() { return N == 2048 && MODE != PASS_INIT ? LMA_KMW_2048 : 2; }

// Register budget: lengths 5 * 2^a are held to two wavefronts per SIMD (at most 256 VGPRs;
// unlimited they take 280-310 and run one wavefront per SIMD, measured 30 % slower at 640);
// the others are not limited.
#ifndef LMA_MIN_WAVES_512
#define LMA_MIN_WAVES_512 1
#endif
template <int N, int MODE>
constexpr int pass_min_waves() {
  if (fft_odd(N) == 5) return 2;
  if (N == 512 && (MODE == PASS_ROW || MODE == PASS_COL)) return LMA_MIN_WAVES_512;
  return 1;
}
// PR (row passes of 512 and 64 points): positions [3N/8, 5N/8) of every line are zeros on the
// way in and not stored on the way out, so the inverse transform takes them as zeros and the
// forward one does not form them
template <int N, int TW, int MODE, int SCHED = 0, int PR = 0>
__global__ __launch_bounds__((PassCfg<N, TW, pass_waves<MODE>(), pass_kmw<N, MODE>()>::WAVES * 64))
__attribute__((amdgpu_waves_per_eu(pass_min_waves<N, MODE>(), 8))) void k_pass(PassArgs a) {
  using C = PassCfg<N, TW, pass_waves<MODE>(), pass_kmw<N, MODE>(), SCHED>;
  constexpr int T = C::T, S = C::S, RS = pass_rows(MODE) ? C::RS_ROW : C::RS_COL, TPB = C::TPB, RPW = C::RPW;
  constexpr int NT = C::WAVES * 64;
  constexpr bool ROWS = pass_rows(MODE);
  constexpr int TOTAL = TW * N;                            // elements of one work item
  constexpr int EPT = TOTAL / NT;                          // per thread
#ifndef LMA_PREFETCH
#define LMA_PREFETCH 1
#endif
// The next item's loads are issued in the item's last round, after its table values have
// been used: a wait for the table also waits for every vector-memory operation issued before
// it, which would otherwise hold each line's transform until the whole prefetch had arrived
// from HBM (and the prefetch registers are free in the rounds before).
#ifndef LMA_LATE_PREFETCH
#define LMA_LATE_PREFETCH 1
#endif
#ifndef LMA_EARLY_TABLE
#define LMA_EARLY_TABLE 1
#endif
#ifndef LMA_ENTRY_STORES_ROW
#define LMA_ENTRY_STORES_ROW 1
#endif
#ifndef LMA_ENTRY_STORES_COL
#define LMA_ENTRY_STORES_COL 0
#endif
  // measured on the 512-point passes: the late prefetch pays in row and column passes and not
  // in the gather (no write-back to overlap with), the entry stores in row passes only
  constexpr bool kLate = LMA_LATE_PREFETCH && MODE != PASS_GATHER && MODE != PASS_REDUCE && MODE != PASS_INIT;
  constexpr bool kEntryStores = kLate && (ROWS ? LMA_ENTRY_STORES_ROW : LMA_ENTRY_STORES_COL);

  constexpr bool PREF = LMA_PREFETCH && EPT <= 16;         // next item prefetched into registers
  constexpr int CHUNK = stage_chunk(EPT);                  // staging step otherwise
  static_assert(TOTAL % NT == 0, "work item must split evenly over the threads");
  __shared__ float2 tile[(TW + (C::WL ? 1 : 0)) * RS];     // extra line: scratch of idle lanes
  // Row and column passes: the item's TW lines of the table (t_j, or the propagator) held in
  // LDS while the workgroup's consecutive items share them (in the XCD-contiguous walk a
  // workgroup takes runs of one tile row or column over several waves), read back by each
  // round instead of from L2
#ifndef LMA_ROW_TAB_LDS
#define LMA_ROW_TAB_LDS 1
#endif
#ifndef LMA_COL_TAB_LDS
#define LMA_COL_TAB_LDS 0   // the column pass measured the same either way (269.1 / 269.6 us)
#endif
  constexpr bool kTabLds = ((LMA_ROW_TAB_LDS && MODE == PASS_ROW) || (LMA_COL_TAB_LDS && MODE == PASS_COL)) && PREF &&
                           N == 512 && TW == 8;
  [[maybe_unused]] __shared__ float2 ttab[kTabLds ? TW * N : 1];
  [[maybe_unused]] int tab_g = -1;                         // tile row whose t_j lines ttab holds
  [[maybe_unused]] __shared__ double part[C::WAVES][8];
  // PASS_INIT: exp(-2 pi i my uy / Qy) at every ky of the item's wave, shared by its lines
  // (when the LDS has room next to the tile: not for 2048-point lines in 8 x 8 tiles)
  constexpr bool kYfac = MODE == PASS_INIT && sizeof(tile) + sizeof(part) + (size_t)N * 16 <= 160 * 1024;
  [[maybe_unused]] __shared__ double2 yfac[kYfac ? N : 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int sub = C::WL ? lane / T : 0;                    // transform within the wavefront
  const int j = C::WL ? lane % T : tid % T;                // thread within the transform
  const int tslot = C::WL ? (tid >> 6) * S + sub : tid / T;  // transform slot within the block
  const bool active = !C::WL || sub < S;
  // column-layout passes skip the tile columns [zlo, zhi) of a gap (the band gap; for the
  // initial waves, the input spectrum's gap): item group g' maps to tile column g' below the
  // gap and g' + (zhi - zlo) above it
  constexpr bool kGapItems = MODE == PASS_COL || MODE == PASS_GATHER || MODE == PASS_REDUCE || MODE == PASS_INIT;
  const int gap = kGapItems ? a.zhi - a.zlo : 0;
  const int ngroups = (ROWS ? a.ny : a.nx) / TW - gap;
  const int B = a.B;
  const int ntx = a.nx / TW;
  const ItemWalk walk(B * ngroups);
  auto group_of = [&](int l) -> int {
    const int gg = l / B;
    return (kGapItems && gg >= a.zlo) ? gg + gap : gg;
  };
  // row passes: tile q of a row item lies in a gap. They do not read tile columns [rlo, rhi),
  // which hold zeros (the band gap after a column pass, the input gap after the initial
  // waves); those whose output goes to a column pass do not write the band gap [zlo, zhi)
  // (not PASS_ROW_LAST, which leaves its wave in real space).
  auto in_gap = [&](int c) -> bool {
    if constexpr (ROWS) {
      const int q = c / (TW * TW);
      return q >= a.zlo && q < a.zhi;
    } else {
      return false;
    }
  };
  auto in_rgap = [&](int c) -> bool {
    if constexpr (ROWS) {
      const int q = c / (TW * TW);
      return q >= a.rlo && q < a.rhi;
    } else {
      return false;
    }
  };
  constexpr bool kGapStores = MODE == PASS_ROW || MODE == PASS_ROW_WIN;

  float2 tw[C::NTW];
  tw_load<N, SCHED>(tw, a.tw, j);

  using M = TileMap<N, TW, ROWS>;
  const int stride_q = ntx * M::TT;                        // column items: tile-to-tile stride
  auto item_ptr = [&](int l) -> float2* {
    const int g = group_of(l), w = l % B;
    return a.work + (size_t)w * a.nx * a.ny + M::item_base(g, a.nx);
  };
  [[maybe_unused]] float2 buf[PREF ? EPT : 1];
  constexpr bool kBufferIO = ROWS ? LMA_BUFFER_IO_ROW : LMA_BUFFER_IO_COL;
  // bytes a work item spans in HBM (row item: TW contiguous lines; column item: N / TW tiles)
  const uint32_t item_bytes = (uint32_t)(ROWS ? (size_t)TW * a.nx * 8 : ((size_t)(N / TW - 1) * stride_q + M::TT) * 8);

  // When a wavefront's 64 elements of a step lie in one tile, their offsets are one uniform
  // part per step (held in scalar registers) plus the lane's own 8 bytes times the lane, and a
  // gap tile is skipped by an empty extent for that step rather than by per-lane offsets.
  // Measured on the 512-point passes: 11 of 86 us off the initial waves, 1 us off the column
  // pass, but 9 us onto the row pass and 3 onto the gather, so those keep per-lane offsets.
#ifndef LMA_SPLIT_OFFSETS
#define LMA_SPLIT_OFFSETS 1
#endif
  constexpr bool kSplitOff = kBufferIO && LMA_SPLIT_OFFSETS && (MODE == PASS_COL || MODE == PASS_INIT) &&
                             M::TT % 64 == 0 && NT % 64 == 0;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane_off = lane * 8;
  // step k: the uniform byte offset of this wavefront's elements and their tile q
  auto step_soff = [&](int k, int& q) -> int {
    const int cb = k * NT + wid * 64;
    q = cb / M::TT;
    return ROWS ? cb * 8 : (q * stride_q + cb % M::TT) * 8;
  };

  // extent: the bytes the loads may touch (0: every load reads zero without a memory access)
  auto load_item = [&](int l, uint32_t extent) {
    const float2* src = item_ptr(l);
    memory_phase_begin();
    if constexpr (kSplitOff) {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        int q;
        const int so = step_soff(k, q);
        const bool skip = a.zread && ROWS && q >= a.rlo && q < a.rhi;
        buf[k] = load_item_elem2(item_rsrc(src, skip ? 0u : extent), lane_off, so);
      }
    } else if constexpr (kBufferIO) {
      const __amdgpu_buffer_rsrc_t r = item_rsrc(src, extent);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        int lds, off;
        M::at(k * NT + tid, stride_q, lds, off);
        // a gap element is read at an offset past the item's extent: zero, no memory access,
        // and no branch (every load of the prefetch is issued, so waits on the loads after it
        // are counted exactly)
        if (a.zread && in_rgap(k * NT + tid)) off = kOutOfItem;
        buf[k] = load_item_elem(r, off);
      }
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        int lds, off;
        M::at(k * NT + tid, stride_q, lds, off);
        buf[k] = (a.zread && in_rgap(k * NT + tid)) ? make_float2(0.f, 0.f) : load_stream(src + off);
      }
    }
    memory_phase_end();
  };
  if constexpr (PREF && MODE != PASS_INIT) {
    if (walk.valid(walk.l)) load_item(walk.l, item_bytes);
    // as many stores as an item writes back, to an empty extent (dropped): the loop is then
    // entered with the memory operations its back edge carries, so the waits at its head
    // cover the prefetch alone instead of the previous item's stores as well
    if constexpr (kBufferIO && kEntryStores) {
      const __amdgpu_buffer_rsrc_t r0 = item_rsrc(a.work, 0u);
#pragma unroll
      for (int k = 0; k < EPT; ++k) store_item_elem2(r0, lane_off, 0, make_float2(0.f, 0.f));
    }
  }
  int next_item = -1;                                      // the item a late prefetch loads
  int cur_item = walk.l;
  auto late_prefetch = [&](int round) {
    if constexpr (PREF && kLate) {
      if (round == RPW - 1) {                              // the last round: the prefetch
                                                           // registers are free until then
        // keep the loads after the table's uses: hoisted above them, they would share its wait
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (kBufferIO) {
          // issued on every path, past the last item with an empty extent: the waits on the
          // loads before them then count these too, and need not cover all of them
          const bool more = next_item >= 0;
          load_item(more ? next_item : cur_item, more ? item_bytes : 0u);
        } else if (next_item >= 0) {
          load_item(next_item, item_bytes);
        }
      }
    }
  };

#pragma unroll 1
  for (int l = walk.l; walk.valid(l); l += walk.step) {
    const int g = group_of(l), w = l % B;
    float2* item = item_ptr(l);
    next_item = walk.valid(l + walk.step) ? l + walk.step : -1;
    cur_item = l;
    // the previous item is out of LDS. Passes that stage their items from registers and write
    // them back through the same LDS slots skip this: each slot is read back (for the store)
    // and then restaged by the same thread, and the write-back sits behind the barrier that
    // follows the transforms.
#ifndef LMA_TOP_BARRIER
#define LMA_TOP_BARRIER 0
#endif
    constexpr bool kOwnSlots = PREF && !LMA_TOP_BARRIER &&
                               (MODE == PASS_ROW || MODE == PASS_COL || MODE == PASS_ROW_WIN || MODE == PASS_ROW_LAST);
    if constexpr (!kOwnSlots) __syncthreads();

    // ---- stage the item's lines into LDS, then start loading the next item ----------------
    if constexpr (MODE != PASS_INIT) {
      if constexpr (PREF) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          int lds, off;
          M::at(k * NT + tid, stride_q, lds, off);
          tile[lds] = buf[k];
        }
        if constexpr (kTabLds) {
          // every wavefront has finished the previous item's table product (it precedes the
          // barrier before the write-back)
          if (g != tab_g) {
            const float2* src = a.table + (size_t)g * TW * N;
#pragma unroll
            for (int k = 0; k < TW * N / NT; ++k) ttab[k * NT + tid] = src[k * NT + tid];
            tab_g = g;
          }
        }
        __syncthreads();
        if (!kLate && walk.valid(l + walk.step)) load_item(l + walk.step, item_bytes);
      } else {
#pragma unroll 1
        for (int c0 = 0; c0 < TOTAL; c0 += NT * CHUNK) {
          float2 st[CHUNK];
#pragma unroll
          for (int k = 0; k < CHUNK; ++k) {
            int lds, off;
            M::at(c0 + k * NT + tid, stride_q, lds, off);
            st[k] = (a.zread && in_rgap(c0 + k * NT + tid)) ? make_float2(0.f, 0.f) : load_stream(item + off);
          }
#pragma unroll
          for (int k = 0; k < CHUNK; ++k) {
            int lds, off;
            M::at(c0 + k * NT + tid, stride_q, lds, off);
            tile[lds] = st[k];
          }
        }
        __syncthreads();
      }
    }

    if constexpr (kYfac) {
      // the translate modulation factors over ky: one FP64 phase per position, reduced exactly
      // in lattice units (my uy mod Qy), for all the item's lines
      const int64_t uy = a.wave_u[2 * w + 1];
      for (int i = tid; i < N; i += NT) {
        const int64_t ay = (((int64_t)freq_index(i, N) * uy) % a.Qy + a.Qy) % a.Qy;
        double sn, cs;
        sincospi(-2.0 * (double)ay / (double)a.Qy, &sn, &cs);
        yfac[i] = make_double2(cs, sn);
      }
      __syncthreads();
    }

    [[maybe_unused]] double acc[8];
    if constexpr (MODE == PASS_REDUCE) {
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    }

#pragma unroll 1
    for (int rr = 0; rr < RPW; ++rr) {
      const int r = rr * TPB + (active ? tslot : 0);       // line within the workgroup
      const int line = g * TW + r;                          // y (row pass) or x (column passes)
      const Slot slot{tile + (active ? r : TW) * RS};
      const float2* tab_base = a.table;
      if constexpr (MODE == PASS_ROW) {
        if (a.wave_spec) tab_base = a.spec_table[a.wave_spec[w]] + a.slice_off;
      }
      const float2* tab = tab_base + (size_t)line * N;
      float2 v[C::E];
      if constexpr (MODE == PASS_INIT) {
        // u(. - pos_w): spectrum times exp(-2 pi i mx ux / Qx) exp(-2 pi i my uy / Qy), each
        // phase reduced exactly in lattice units and evaluated in FP64, their product in FP64;
        // lines are kx, positions ky
        const int mx = freq_index(line, a.nx);
        const int64_t ux = a.wave_u[2 * w];
        const int64_t ax = (((int64_t)mx * ux) % a.Qx + a.Qx) % a.Qx;
        double xs, xc;
        sincospi(-2.0 * (double)ax / (double)a.Qx, &xs, &xc);
#pragma unroll
        for (int m = 0; m < C::E; ++m) {
          const int ky = j + T * m;
          double2 yf;
          if constexpr (kYfac) {
            yf = yfac[ky];
          } else {
            const int64_t ay = (((int64_t)freq_index(ky, N) * a.wave_u[2 * w + 1]) % a.Qy + a.Qy) % a.Qy;
            sincospi(-2.0 * (double)ay / (double)a.Qy, &yf.y, &yf.x);
          }
          const double cs = xc * yf.x - xs * yf.y, sn = xc * yf.y + xs * yf.x;
          v[m] = cmul(tab[ky], make_float2((float)cs, (float)sn));
        }
        fft<N, +1, C::WL, 0, 0, SCHED>(v, j, tw, a.tw, slot);
      } else {
        // column-type passes of 512 or 64 points prune their transforms where the propagator
        // vanishes (the row pass would prune the band gap the same way, but measured 5 % slower
        // with it: its two code paths cost more than the skipped work)
        constexpr bool kPrunable = fft_prunable(N) && (MODE == PASS_COL || MODE == PASS_GATHER || MODE == PASS_REDUCE);
        const bool prune = kPrunable && a.prune;
        // the line's table values (t_j or the propagator), loaded before the first transform so
        // that it covers their latency (measured on the 512-point passes: 4 % off the row pass,
        // neutral in the column pass, 8 % slower in the gather, which has no write-back)
        constexpr bool kEarly = LMA_EARLY_TABLE && (MODE == PASS_ROW || MODE == PASS_COL);
        [[maybe_unused]] float2 tv[kEarly ? C::E : 1];
        if constexpr (kEarly) {
#pragma unroll
          for (int m = 0; m < C::E; ++m) {
            if constexpr (kTabLds) tv[m] = ttab[r * N + j + T * m];
            else tv[m] = tab[j + T * m];
          }
        }
        auto tab_at = [&](int m) -> float2 {
          if constexpr (kEarly) return tv[m];
          else return tab[j + T * m];
        };
#pragma unroll
        for (int m = 0; m < C::E; ++m) v[m] = slot.get(j + T * m);
        // the first stage overwrites the line: every thread of the transform must have read it
        exchange_sync<C::WL>();
        if constexpr (MODE == PASS_ROW) {
          fft<N, +1, C::WL, 0, PR ? PRUNE_IN : 0, SCHED>(v, j, tw, a.tw, slot);
#pragma unroll
          for (int m = 0; m < C::E; ++m) v[m] = cmul(v[m], tab_at(m));
          late_prefetch(rr);
          fft<N, -1, C::WL, 0, PR ? PRUNE_OUT : 0, SCHED>(v, j, tw, a.tw, slot);
        } else if constexpr (MODE == PASS_ROW_WIN || MODE == PASS_ROW_LAST) {
          fft<N, +1, C::WL, 0, 0, SCHED>(v, j, tw, a.tw, slot);
          // the cell's transmission at the window: row (y0 + line) mod tny, columns
          // (x0 + x) mod tnx with (x0, y0) the window origin of wave w (exact integers)
          const int64_t px = a.wave_u[2 * w] * a.tnx / a.Qx, py = a.wave_u[2 * w + 1] * a.tny / a.Qy;
          int ry = (int)((py - a.hy + line) % a.tny);
          if (ry < 0) ry += a.tny;
          int bx = (int)((px - a.hx) % a.tnx);
          if (bx < 0) bx += a.tnx;
          const float2* trow = a.table + (size_t)ry * a.tnx;
#pragma unroll
          for (int m = 0; m < C::E; ++m) {
            int col = bx + j + T * m;
            if (col >= a.tnx) col -= a.tnx;
            v[m] = cmul(v[m], trow[col]);
          }
          late_prefetch(rr);
          if constexpr (MODE == PASS_ROW_WIN) fft<N, -1, C::WL, 0, 0, SCHED>(v, j, tw, a.tw, slot);
        } else {
          // column FFT, propagator; with pruning the outputs in [3N/8, 5N/8), where the
          // propagator vanishes for every column, are not formed and stay zeros
          bool pruned = false;
          if constexpr (kPrunable) {
            if (prune) {
              fft<N, -1, C::WL, 0, PRUNE_OUT, SCHED>(v, j, tw, a.tw, slot);
#pragma unroll
              for (int m = 0; m < C::E; ++m)
                v[m] = (m == 3 || m == 4) ? make_float2(0.f, 0.f) : cmul(v[m], tab_at(m));
              pruned = true;
            }
          }
          if (!pruned) {
            fft<N, -1, C::WL, 0, 0, SCHED>(v, j, tw, a.tw, slot);
#pragma unroll
            for (int m = 0; m < C::E; ++m) v[m] = cmul(v[m], tab_at(m));
          }
          late_prefetch(rr);
          if constexpr (MODE == PASS_COL) {
            if constexpr (kPrunable) {
              if (prune) fft<N, +1, C::WL, 0, PRUNE_IN, SCHED>(v, j, tw, a.tw, slot);
              else fft<N, +1, C::WL, 0, 0, SCHED>(v, j, tw, a.tw, slot);
            } else {
              fft<N, +1, C::WL, 0, 0, SCHED>(v, j, tw, a.tw, slot);
            }
          } else if constexpr (MODE == PASS_GATHER) {
            if (active) {
              const int64_t brow = a.wave_row[w];
              const int32_t* cm = a.comp + (size_t)line * N;
#pragma unroll
              for (int m = 0; m < C::E; ++m) {
                const int d = cm[j + T * m];
                if (d >= 0) {
                  if (a.split_bf16) {
                    __hip_bfloat16 q[4];
                    split_bf16(v[m].x, q[0], q[1]);
                    split_bf16(v[m].y, q[2], q[3]);
                    reinterpret_cast<uint2*>(a.basis)[brow * a.D + d] = *reinterpret_cast<uint2*>(q);
                  } else {
                    reinterpret_cast<float2*>(a.basis)[brow * a.D + d] = v[m];
                  }
                }
              }
            }
          } else if constexpr (MODE == PASS_REDUCE) {
            if (active) {
              const uint32_t* mk = a.mask + (size_t)line * N;
#pragma unroll
              for (int m = 0; m < C::E; ++m) {
                const uint32_t bits = mk[j + T * m];
                const double p = (double)v[m].x * v[m].x + (double)v[m].y * v[m].y;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                  if (bits & (1u << q)) acc[q] += p;
              }
            }
          }
        }
      }
      if constexpr (MODE == PASS_ROW || MODE == PASS_COL || MODE == PASS_INIT || MODE == PASS_ROW_WIN ||
                    MODE == PASS_ROW_LAST) {
        if (active) {
#pragma unroll
          for (int m = 0; m < C::E; ++m) slot.put(j + T * m, v[m]);
        }
      }
    }

    if constexpr (MODE == PASS_REDUCE) {
      // ring sums of this item: wavefront shuffles, then one partial per wavefront
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        double x = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) part[tid >> 6][q] = x;
      }
      __syncthreads();
      if (tid < a.ndet) {
        double sum = 0.0;
        for (int i = 0; i < C::WAVES; ++i) sum += part[i][tid];
        atomicAdd(a.img + tid * a.img_stride + a.wave_row[w], sum * a.scale);
      }
    } else if constexpr (MODE != PASS_GATHER) {
      // ---- write the lines back, whole tiles, in place ------------------------------------
      __syncthreads();
      memory_phase_begin();
      if constexpr (kSplitOff) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          int lds, off, q;
          M::at(k * NT + tid, stride_q, lds, off);
          const int so = step_soff(k, q);
          const bool skip = kGapStores && q >= a.zlo && q < a.zhi;
          store_item_elem2(item_rsrc(item, skip ? 0u : item_bytes), lane_off, so, tile[lds]);
        }
      } else if constexpr (kBufferIO) {
        const __amdgpu_buffer_rsrc_t r = item_rsrc(item, item_bytes);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          int lds, off;
          M::at(k * NT + tid, stride_q, lds, off);
          if (kGapStores && in_gap(k * NT + tid)) off = kOutOfItem;
          store_item_elem(r, off, tile[lds]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          int lds, off;
          M::at(k * NT + tid, stride_q, lds, off);
          if (!kGapStores || !in_gap(k * NT + tid)) store_stream(item + off, tile[lds]);
        }
      }
      memory_phase_end();
    }
  }
}

// ------------------------------------------------------------------------------------------
// contraction: psi_hat_p[d] = sum_j alpha_{s(p),j} U_hat[row(p,j)][d], then ring sums
// ------------------------------------------------------------------------------------------
constexpr int kCT = 256;      // threads per block = pixels per chunk

template <int SPLIT>
__device__ __forceinline__ float2 load_basis(const void* basis, int64_t i) {
  if constexpr (SPLIT) {
    uint2 raw = reinterpret_cast<const uint2*>(basis)[i];
    const __hip_bfloat16* q = reinterpret_cast<const __hip_bfloat16*>(&raw);
    return make_float2(__bfloat162float(q[0]) + __bfloat162float(q[1]),
                       __bfloat162float(q[2]) + __bfloat162float(q[3]));
  } else {
    return reinterpret_cast<const float2*>(basis)[i];
  }
}

// OUT: 0 ring sums (2-D STEM), 1 the pattern |psi_hat|^2 at every detector pixel (4-D STEM),
// 2 sums over annuli of scattering angle (3-D STEM)
enum { OUT_RINGS = 0, OUT_PATTERN = 1, OUT_RADIAL = 2 };

template <int SPLIT, int kPT, int OUT>
__global__ __launch_bounds__(kCT) void k_contract(Contraction c) {
  extern __shared__ unsigned char dyn[];
  int64_t* rows = reinterpret_cast<int64_t*>(dyn);                        // [kPT][L]
  float2* al = reinterpret_cast<float2*>(rows + (size_t)kPT * c.L);       // [kPT][L]
  [[maybe_unused]] double* bins = reinterpret_cast<double*>(al + (size_t)kPT * c.L);  // [kPT][nbins]
  __shared__ double part[kCT / 64][kPT];
  const int chunk = blockIdx.x;
  const int p0 = blockIdx.y * kPT;
  const int np = c.probe_list ? c.n_list : c.ww * c.wh;
  const int npb = min(kPT, np - p0);
  for (int i = threadIdx.x; i < npb * c.L; i += kCT) {
    const int pi = i / c.L, jj = i % c.L;
    const int p = c.probe_list ? c.probe_list[p0 + pi] : p0 + pi;
    const int a = c.wa0 + p % c.ww, b = c.wb0 + p / c.ww;
    const int cx = a % c.ncls_x, cy = b % c.ncls_y;
    const int s = cy * c.ncls_x + cx;
    const int shx = (a / c.ncls_x) * c.stepx, shy = (b / c.ncls_y) * c.stepy;
    const int ta = (c.set_dx[s * c.L + jj] + shx) % c.Rfx;
    const int tb = (c.set_dy[s * c.L + jj] + shy) % c.Rfy;
    const int row = c.row_of[tb * c.Rfx + ta];
    // every neighbour of a window probe is resident by construction; a missing row
    // contributes nothing instead of reading outside the basis
    rows[pi * c.L + jj] = row >= 0 ? (int64_t)row * c.D : 0;
    al[pi * c.L + jj] = row >= 0 ? c.alpha[s * c.L + jj] : make_float2(0.f, 0.f);
  }
  if constexpr (OUT == OUT_RADIAL) {
    for (int i = threadIdx.x; i < kPT * c.nbins; i += kCT) bins[i] = 0.0;
  }
  __syncthreads();
  const int start = c.chunk_start[chunk], len = c.chunk_len[chunk];
  const uint32_t mask = c.chunk_mask[chunk];
  const int t = threadIdx.x;
  double val[kPT];
#pragma unroll
  for (int pi = 0; pi < kPT; ++pi) {
    val[pi] = 0.0;
    if (pi < npb && t < len) {
      float2 acc = make_float2(0.f, 0.f);
      const int64_t d = start + t;
      for (int jj = 0; jj < c.L; ++jj) {
        const float2 u = load_basis<SPLIT>(c.basis, rows[pi * c.L + jj] + d);
        const float2 w = al[pi * c.L + jj];
        acc.x += w.x * u.x - w.y * u.y;
        acc.y += w.x * u.y + w.y * u.x;
      }
      val[pi] = (double)acc.x * acc.x + (double)acc.y * acc.y;
    }
  }
  if constexpr (OUT == OUT_PATTERN) {
    if (t < len) {
#pragma unroll
      for (int pi = 0; pi < kPT; ++pi)
        if (pi < npb) {
          const int p = c.probe_list ? c.probe_list[p0 + pi] : p0 + pi;
          c.patterns[(int64_t)p * c.D + start + t] = (float)(val[pi] * c.scale);
        }
    }
    return;
  }
  if constexpr (OUT == OUT_RADIAL) {
    const int bin = t < len ? c.bin_of[start + t] : -1;
    if (bin >= 0) {
#pragma unroll
      for (int pi = 0; pi < kPT; ++pi)
        if (pi < npb) atomicAdd(&bins[pi * c.nbins + bin], val[pi]);
    }
    __syncthreads();
    const int64_t stride = c.probe_list ? c.n_list : (int64_t)c.ww * c.wh;
    for (int i = t; i < npb * c.nbins; i += kCT) {
      const double x = bins[i];
      if (x != 0.0) {
        const int pi = i / c.nbins, b = i % c.nbins;
        const int p = c.probe_list ? c.probe_list[p0 + pi] : p0 + pi;
        atomicAdd(c.radial + (int64_t)b * stride + p, x * c.scale);
      }
    }
    return;
  }
  const int lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int pi = 0; pi < kPT; ++pi) {
    double x = val[pi];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) part[wv][pi] = x;
  }
  __syncthreads();
  if (t < npb) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kCT / 64; ++i) s += part[i][t];
    s *= c.scale;
    const int p = c.probe_list ? c.probe_list[p0 + t] : p0 + t;
    const int64_t stride = (int64_t)c.ww * c.wh;
    for (int r = 0; r < c.ndet; ++r)
      if (mask & (1u << r)) atomicAdd(c.img + (int64_t)r * stride + p, s);
  }
}

// ------------------------------------------------------------------------------------------
// contraction of a whole window as a banded complex GEMM on MFMA (v_mfma_f32_16x16x4f32):
//   C[probe m][pixel n] = sum_k A[m][k] B[k][n]
// A: alpha of the 16 probes of a 4 x 4 sub-block against the K translates of the union of
// their neighbour sets (zero where a translate is not a probe's neighbour), held in registers
// for the whole workgroup; B: the basis rows of the super-tile's translate rectangle at 16
// detector pixels, staged in LDS. Fragment layouts of the 16x16x4 instruction: lane l holds
// A[l % 16][k0 + l / 16] and B[k0 + l / 16][l % 16]; the accumulator holds
// C[4 (l / 16) + r][l % 16], r < 4. Complex products take four real MFMAs:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B.
// ------------------------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Work item of a contraction workgroup: (super-tile, detector-pixel chunk), in chunk-major
// order. Blocks are dispatched round-robin over the 8 XCDs; each XCD takes a contiguous range
// of that order, so the XCDs work on different chunks at once (no basis segment is fetched by
// two XCDs together) and an XCD's consecutive workgroups are neighbouring super-tiles of one
// chunk, whose translate rectangles overlap in its L2.
__device__ __forceinline__ void stencil_item(const Stencil& c, int& ti, int& tj, int& chunk) {
  const int nt = c.tiles_x * c.tiles_y;
#ifndef LMA_CONTRACT_XCD
#define LMA_CONTRACT_XCD 1
#endif
  const int l = LMA_CONTRACT_XCD ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int t = l % nt;
  chunk = l / nt;
  ti = c.tile_x0 + t % c.tiles_x;
  tj = c.tile_y0 + t / c.tiles_x;
}

template <int SPLIT, int KS>
__global__ __launch_bounds__(256) void k_contract_mfma(Stencil c) {
  extern __shared__ unsigned char dyn[];
  const int nt = c.W * c.H;
  float2* slab = reinterpret_cast<float2*>(dyn);                          // [nt][16]
  int32_t* rowid = reinterpret_cast<int32_t*>(slab + (size_t)nt * 16);    // [nt]
  int ti, tj, chunk;
  stencil_item(c, ti, tj, chunk);
  const int ox = (c.ox0 + ti * c.tile_dx) % c.Rfx;
  const int oy = (c.oy0 + tj * c.tile_dy) % c.Rfy;
  for (int t = threadIdx.x; t < nt; t += 256) {
    const int x = t % c.W, y = t / c.W;
    rowid[t] = c.row_of[((oy + y) % c.Rfy) * c.Rfx + (ox + x) % c.Rfx];
  }
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int kk = lane >> 4, n = lane & 15;
  float2 A[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) A[ks] = ks < c.nks ? c.a[ks * 64 + lane] : make_float2(0.f, 0.f);
  // the K-step offsets one per lane (steps 64 and up in a second register), read into scalar
  // registers by each step rather than loaded from memory there
  static_assert(KS <= 128, "two offsets per lane");
  const int koff0 = lane < c.nks ? c.ks_off[lane] : 0;
  const int koff1 = KS > 64 && 64 + lane < c.nks ? c.ks_off[64 + lane] : 0;
  // rectangle index of this lane's B element at K-step ks is base + ks_off[ks]
  const int base = (wv >> 1) * c.sub_dy * c.W + (wv & 1) * c.sub_dx + kk;
  const int start = c.chunk_start[chunk], len = c.chunk_len[chunk];
  const uint32_t mask = c.chunk_mask[chunk];
  double val[4] = {0.0, 0.0, 0.0, 0.0};
  for (int d0 = 0; d0 < len; d0 += 16) {
    __syncthreads();  // row ids written, previous slab consumed
    const int rem = len - d0;
    // fill the slab with kFill loads in flight per thread
    constexpr int kFill = 8;
    for (int i0 = threadIdx.x; i0 < nt * 16; i0 += 256 * kFill) {
      float2 v[kFill];
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        const int i = i0 + u * 256;
        v[u] = make_float2(0.f, 0.f);
        if (i < nt * 16) {
          const int t = i >> 4, q = i & 15;
          const int r = rowid[t];
          // a translate the window does not need is not resident: it only meets zero coefficients
          if (r >= 0 && q < rem) v[u] = load_basis<SPLIT>(c.basis, (int64_t)r * c.D + start + d0 + q);
        }
      }
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        const int i = i0 + u * 256;
        if (i < nt * 16) slab[i] = v[u];
      }
    }
    __syncthreads();
    f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
    // runs of four K-steps under one uniform test; steps past the last multiply zero A
    // fragments by the slab's first rows and add exact zeros
#pragma unroll
    for (int kb = 0; kb < KS; kb += 4) {
      if (kb < c.nks) {
#pragma unroll
        for (int ks = kb; ks < kb + 4 && ks < KS; ++ks) {
          const int o = ks < 64 ? __builtin_amdgcn_readlane(koff0, ks) : __builtin_amdgcn_readlane(koff1, ks - 64);
          const float2 b = slab[(base + o) * 16 + n];
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ks].x, b.x, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ks].x, b.y, cim, 0, 0, 0);
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-A[ks].y, b.y, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ks].y, b.x, cim, 0, 0, 0);
        }
      }
    }
    if (n < rem) {
#pragma unroll
      for (int r = 0; r < 4; ++r) val[r] += (double)cre[r] * cre[r] + (double)cim[r] * cim[r];
    }
  }
  // ring sum over the 16 pixel lanes of each probe row
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double x = val[r];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o);
    val[r] = x;
  }
  if (n == 0) {
    const int by = tj * 8 + (wv >> 1) * 4 + kk;
    const int64_t stride = (int64_t)c.ww * c.wh;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int bx = ti * 8 + (wv & 1) * 4 + r;
      if (bx >= c.pa0 && bx < c.pa1 && by >= c.pb0 && by < c.pb1) {
        const double v = val[r] * c.scale;
        for (int d = 0; d < c.ndet; ++d)
          if (mask & (1u << d)) atomicAdd(c.img + (int64_t)d * stride + (int64_t)by * c.ww + bx, v);
      }
    }
  }
}

__global__ void k_fill_zero(double* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 0.0;
}

__global__ void k_scale_out(double* out, const double* img, int64_t n, double w, int acc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (acc ? out[i] : 0.0) + w * img[i];
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
bool supported(int nx, int ny) { return fft_length_ok(nx) && fft_length_ok(ny); }

hipError_t transmission(const float* v, float2* t, int64_t n, double sigma, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  k_transmission<<<(unsigned)((n + th - 1) / th), th, 0, s>>>(v, t, n, sigma);
  return hipGetLastError();
}

// host-side caches below are filled on first use by any thread (same value from each)
static int device_cus() {
  static std::atomic<int> cached{0};
  int cus = cached.load(std::memory_order_relaxed);
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cached.store(cus, std::memory_order_relaxed);
  }
  return cus;
}

// lengths built with the other radix schedules as well (those with unequal radices whose
// passes take measurable time), in 4 x 4 and 8 x 8 tiles
__host__ __device__ constexpr bool sched_variants(int n, int tw) {
  return (tw == 4 || tw == 8) && (n == 256 || n == 384 || n == 640 || n == 1024 || n == 2048);
}
template <int N, int TW, int MODE, int SCHED, int PR = 0>
static hipError_t pass_launch_s(const PassArgs& a0, int lines, int B, hipStream_t s) {
  if (lines % TW) return hipErrorInvalidValue;
  constexpr int threads = PassCfg<N, TW, pass_waves<MODE>(), pass_kmw<N, MODE>(), SCHED>::WAVES * 64;
  static std::atomic<int> cached{0};   // workgroups of this kernel resident per CU
  int resident = cached.load(std::memory_order_relaxed);
  if (resident == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, (const void*)k_pass<N, TW, MODE, SCHED, PR>, threads, 0) !=
            hipSuccess ||
        resident <= 0)
      resident = 1;
    cached.store(resident, std::memory_order_relaxed);
  }
  PassArgs a = a0;
  a.B = B;
  if (a.zlo < 0 || a.zhi < a.zlo || a.zhi > a.nx / TW || a.rlo < 0 || a.rhi < a.rlo || a.rhi > a.nx / TW)
    return hipErrorInvalidValue;
  constexpr bool kGapItems = MODE == PASS_COL || MODE == PASS_GATHER || MODE == PASS_REDUCE || MODE == PASS_INIT;
  const int64_t items = (int64_t)B * (lines / TW - (kGapItems ? a.zhi - a.zlo : 0));
  if (items <= 0) return hipSuccess;
  int64_t grid = std::min<int64_t>(items, (int64_t)resident * device_cus());
  if (grid >= 8) grid &= ~(int64_t)7;
  k_pass<N, TW, MODE, SCHED, PR><<<(unsigned)grid, threads, 0, s>>>(a);
  return hipGetLastError();
}
// the schedule a length takes unless one is asked for: 640 points run 25-29 % faster with the
// radix-5 stage last (row and column passes, 512-wave launches); the other lengths are fastest
// in the base order or within 4 % of it
__host__ __device__ constexpr int default_sched(int n) { return n == 640 ? 2 : 0; }
template <int N, int TW, int MODE>
static hipError_t pass_launch(const PassArgs& a, int lines, int B, hipStream_t s, int sched) {
  if (sched < 0) sched = default_sched(N);
  if constexpr (sched_variants(N, TW)) {
    if (sched == 1) return pass_launch_s<N, TW, MODE, 1>(a, lines, B, s);
    if (sched == 2) return pass_launch_s<N, TW, MODE, 2>(a, lines, B, s);
  }
  if constexpr (MODE == PASS_ROW && fft_prunable(N) && LMA_PRUNE_ROWS) {
    // the zeros read (tile columns [rlo, rhi)) and the columns not stored ([zlo, zhi)) both
    // cover [3N/8, 5N/8)
    const bool in = a.zread && a.rlo * TW <= 3 * N / 8 && a.rhi * TW >= 5 * N / 8;
    const bool out = a.zlo * TW <= 3 * N / 8 && a.zhi * TW >= 5 * N / 8;
    if (in && out) return pass_launch_s<N, TW, MODE, 0, 1>(a, lines, B, s);
  }
  return pass_launch_s<N, TW, MODE, 0>(a, lines, B, s);
}

template <int MODE>
static hipError_t pass_dispatch(int N, int TW, int lines, const PassArgs& a, int B, hipStream_t s, int sched = -1) {
  if (TW == 16) {
    switch (N) {
      case 16: return pass_launch<16, 16, MODE>(a, lines, B, s, sched);
      case 32: return pass_launch<32, 16, MODE>(a, lines, B, s, sched);
      case 64: return pass_launch<64, 16, MODE>(a, lines, B, s, sched);
      case 128: return pass_launch<128, 16, MODE>(a, lines, B, s, sched);
      case 256: return pass_launch<256, 16, MODE>(a, lines, B, s, sched);
      case 512: return pass_launch<512, 16, MODE>(a, lines, B, s, sched);
    }
  } else if (TW == 4) {
    switch (N) {
      case 16: return pass_launch<16, 4, MODE>(a, lines, B, s, sched);
      case 32: return pass_launch<32, 4, MODE>(a, lines, B, s, sched);
      case 64: return pass_launch<64, 4, MODE>(a, lines, B, s, sched);
      case 128: return pass_launch<128, 4, MODE>(a, lines, B, s, sched);
      case 256: return pass_launch<256, 4, MODE>(a, lines, B, s, sched);
      case 512: return pass_launch<512, 4, MODE>(a, lines, B, s, sched);
      case 1024: return pass_launch<1024, 4, MODE>(a, lines, B, s, sched);
      case 2048: return pass_launch<2048, 4, MODE>(a, lines, B, s, sched);
      case 96: return pass_launch<96, 4, MODE>(a, lines, B, s, sched);
      case 192: return pass_launch<192, 4, MODE>(a, lines, B, s, sched);
      case 384: return pass_launch<384, 4, MODE>(a, lines, B, s, sched);
      case 640: return pass_launch<640, 4, MODE>(a, lines, B, s, sched);
    }
  } else if (TW == 8) {
    switch (N) {
      case 16: return pass_launch<16, 8, MODE>(a, lines, B, s, sched);
      case 32: return pass_launch<32, 8, MODE>(a, lines, B, s, sched);
      case 64: return pass_launch<64, 8, MODE>(a, lines, B, s, sched);
      case 128: return pass_launch<128, 8, MODE>(a, lines, B, s, sched);
      case 256: return pass_launch<256, 8, MODE>(a, lines, B, s, sched);
      case 512: return pass_launch<512, 8, MODE>(a, lines, B, s, sched);
      case 1024: return pass_launch<1024, 8, MODE>(a, lines, B, s, sched);
      case 2048: return pass_launch<2048, 8, MODE>(a, lines, B, s, sched);
      case 96: return pass_launch<96, 8, MODE>(a, lines, B, s, sched);
      case 192: return pass_launch<192, 8, MODE>(a, lines, B, s, sched);
      case 384: return pass_launch<384, 8, MODE>(a, lines, B, s, sched);
      case 640: return pass_launch<640, 8, MODE>(a, lines, B, s, sched);
    }
  }
  return hipErrorInvalidValue;
}

// 8 x 8 tiles (512 B) keep the LDS tile of a workgroup at ~41 KB for 512-point lines, so several
// workgroups share a CU; grids with a side above 512 use 4 x 4 tiles (128 B), which halve the
// LDS tile and prefetch registers of the long-line workgroups (measured +28 % at 1024^2);
// 16 x 16 tiles (2 KB) measured slower and need N <= 512.
static std::atomic<int> g_tile_width{0};   // 0: default; 4, 8 or 16 forces a tile width (tuning)
void set_tile_width(int tw) { g_tile_width.store((tw == 4 || tw == 8 || tw == 16) ? tw : 0); }
int radix_schedules(int nx, int ny, int tw) { return sched_variants(nx, tw) || sched_variants(ny, tw) ? 3 : 1; }
int tile_width(int nx, int ny) {
  const int forced = g_tile_width.load();
  if (nx > 512 || ny > 512) return forced == 8 ? 8 : 4;
  return forced ? forced : 8;
}

bool tile_width_ok(int nx, int ny, int tw) {
  auto side = [tw](int n) {
    if (n % tw) return false;
    if (tw == 16) return fft_pow2(n) && n <= 512;
    return tw == 4 || tw == 8;
  };
  return fft_length_ok(nx) && fft_length_ok(ny) && side(nx) && side(ny);
}
static int tw_of(const Tables& T) { return T.tw ? T.tw : tile_width(T.nx, T.ny); }

static PassArgs pass_args(const Tables& T, float2* work) {
  PassArgs a{};
  a.work = work;
  a.nx = T.nx;
  a.ny = T.ny;
  a.Qx = T.Qx;
  a.Qy = T.Qy;
  // tile columns wholly inside the band gap
  const int tw = tw_of(T);
  const int lo = (T.zc0 + tw - 1) / tw, hi = T.zc1 / tw;
  if (T.zc0 >= 0 && T.zc1 <= T.nx && hi > lo) {
    a.zlo = a.rlo = lo;
    a.zhi = a.rhi = hi;
  }
  a.prune = LMA_PRUNE && T.prop_z34 && fft_prunable(T.ny) ? 1 : 0;   // column-type passes
  return a;
}
// tile columns wholly inside the input spectrum's gap
static void input_gap_tiles(const Tables& T, int* lo, int* hi) {
  const int tw = tw_of(T);
  *lo = (T.ic0 + tw - 1) / tw;
  *hi = T.ic1 / tw;
  if (T.ic0 < 0 || T.ic1 > T.nx || *hi <= *lo) *lo = *hi = 0;
}

hipError_t init_waves(const Tables& T, float2* work, const int64_t* wave_u, int B, hipStream_t s) {
  PassArgs a = pass_args(T, work);
  input_gap_tiles(T, &a.zlo, &a.zhi);   // items skipped: the spectrum vanishes there
  a.rlo = a.rhi = 0;
  a.table = T.specT;
  a.tw = T.twy;
  a.wave_u = wave_u;
  return pass_dispatch<PASS_INIT>(T.ny, tw_of(T), T.nx, a, B, s, T.sched);
}

hipError_t row_pass(const Tables& T, float2* work, const float2* trans_j, int B, bool after_column, hipStream_t s) {
  PassArgs a = pass_args(T, work);
  if (!after_column) input_gap_tiles(T, &a.rlo, &a.rhi);   // the initial waves skipped these
  a.zread = 1;
  a.prune = 0;
  a.table = trans_j;
  a.tw = T.twx;
  return pass_dispatch<PASS_ROW>(T.nx, tw_of(T), T.ny, a, B, s, T.sched);
}

hipError_t row_pass_specimens(const Tables& T, float2* work, const float2* const* spec_trans, const int32_t* wave_spec,
                              int64_t slice_off, int B, bool after_column, hipStream_t s) {
  PassArgs a = pass_args(T, work);
  if (!after_column) input_gap_tiles(T, &a.rlo, &a.rhi);
  a.zread = 1;
  a.prune = 0;
  a.table = nullptr;
  a.spec_table = spec_trans;
  a.wave_spec = wave_spec;
  a.slice_off = slice_off;
  a.tw = T.twx;
  return pass_dispatch<PASS_ROW>(T.nx, tw_of(T), T.ny, a, B, s, T.sched);
}

hipError_t row_pass_window(const Tables& Tw, float2* work, const float2* trans_j, int cell_nx, int cell_ny,
                           const int64_t* wave_u, int64_t Qx, int64_t Qy, bool last, bool after_column, int B,
                           hipStream_t s) {
  PassArgs a = pass_args(Tw, work);
  if (!after_column) input_gap_tiles(Tw, &a.rlo, &a.rhi);
  a.zread = 1;
  a.table = trans_j;
  a.tw = Tw.twx;
  a.wave_u = wave_u;
  a.Qx = Qx;
  a.Qy = Qy;
  a.tnx = cell_nx;
  a.tny = cell_ny;
  a.hx = Tw.nx / 2;
  a.hy = Tw.ny / 2;
  return last ? pass_dispatch<PASS_ROW_LAST>(Tw.nx, tw_of(Tw), Tw.ny, a, B, s, Tw.sched)
              : pass_dispatch<PASS_ROW_WIN>(Tw.nx, tw_of(Tw), Tw.ny, a, B, s, Tw.sched);
}

// ------------------------------------------------------------------------------------------
// the last step of windowed waves: each window's real-space wave is placed in the cell at its
// window (zero elsewhere, periodic) and row-transformed on the cell's grid, which leaves the
// mixed domain (x frequency, y spatial) that the gather pass takes. One block per (cell row,
// wave), one transform of N = nx points.
// ------------------------------------------------------------------------------------------
struct EmbedArgs {
  float2* out;               // [B][cell tiles], cell tile width TW
  const float2* win;         // [B][window tiles], window tile width wtw
  int nx, ny;                // cell
  int wnx, wny, wtw;         // window
  const int64_t* wave_u;     // [B][2] positions in lattice units
  int64_t Qx, Qy;
  const float2* twx;         // cell twiddles exp(-2 pi i t / nx)
};

template <int N, int TW>
__global__ __launch_bounds__(N / fft_elems(N)) void k_embed(EmbedArgs a) {
  constexpr int E = fft_elems(N), T = N / E;
  constexpr bool WL = T <= 64;
  __shared__ float2 line[slot_pos(N - 1) + 1];
  const int y = (int)(blockIdx.x % (unsigned)a.ny), w = (int)(blockIdx.x / (unsigned)a.ny);
  const int j = threadIdx.x;
  float2 tw[tw_count(N)];
  tw_load<N>(tw, a.twx, j);
  const int64_t px = a.wave_u[2 * w] * a.nx / a.Qx, py = a.wave_u[2 * w + 1] * a.ny / a.Qy;
  int wy = (int)((y - (py - a.wny / 2)) % a.ny);        // window row of cell row y
  if (wy < 0) wy += a.ny;
  int x0 = (int)((px - a.wnx / 2) % a.nx);              // cell column of window column 0
  if (x0 < 0) x0 += a.nx;
  const bool inside = wy < a.wny;                        // uniform over the block
  const float2* src = a.win + (size_t)w * a.wnx * a.wny;
  const int wt = a.wtw, wtiles = a.wnx / wt;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int x = j + T * m;
    int wx = x - x0;
    if (wx < 0) wx += a.nx;
    v[m] = make_float2(0.f, 0.f);
    if (inside && wx < a.wnx)
      v[m] = src[((size_t)(wy / wt) * wtiles + wx / wt) * wt * wt + (wy % wt) * wt + wx % wt];
  }
  if (inside) fft<N, -1, WL, 1>(v, j, tw, a.twx, Slot{line});
  float2* dst = a.out + (size_t)w * a.nx * a.ny;
  const int ctiles = a.nx / TW;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int x = j + T * m;
    dst[((size_t)(y / TW) * ctiles + x / TW) * TW * TW + (y % TW) * TW + x % TW] = v[m];
  }
}

template <int N, int TW>
static hipError_t embed_launch(const EmbedArgs& a, int B, hipStream_t s) {
  k_embed<N, TW><<<(unsigned)((int64_t)B * a.ny), N / fft_elems(N), 0, s>>>(a);
  return hipGetLastError();
}

template <int TW>
static hipError_t embed_dispatch(const EmbedArgs& a, int B, hipStream_t s) {
  switch (a.nx) {
    case 16: return embed_launch<16, TW>(a, B, s);
    case 32: return embed_launch<32, TW>(a, B, s);
    case 64: return embed_launch<64, TW>(a, B, s);
    case 96: return embed_launch<96, TW>(a, B, s);
    case 128: return embed_launch<128, TW>(a, B, s);
    case 192: return embed_launch<192, TW>(a, B, s);
    case 256: return embed_launch<256, TW>(a, B, s);
    case 384: return embed_launch<384, TW>(a, B, s);
    case 512: return embed_launch<512, TW>(a, B, s);
    case 640: return embed_launch<640, TW>(a, B, s);
    case 1024: return embed_launch<1024, TW>(a, B, s);
    case 2048: return embed_launch<2048, TW>(a, B, s);
  }
  return hipErrorInvalidValue;
}

hipError_t embed_windows(const Tables& T, float2* work, const Tables& Tw, const float2* win, const int64_t* wave_u,
                         int B, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  EmbedArgs a{};
  a.out = work;
  a.win = win;
  a.nx = T.nx;
  a.ny = T.ny;
  a.wnx = Tw.nx;
  a.wny = Tw.ny;
  a.wtw = tw_of(Tw);
  a.wave_u = wave_u;
  a.Qx = T.Qx;
  a.Qy = T.Qy;
  a.twx = T.twx;
  const int tw = tw_of(T);
  if (a.wnx > a.nx || a.wny > a.ny || a.wnx % a.wtw || a.wny % a.wtw) return hipErrorInvalidValue;
  if (tw == 4) return embed_dispatch<4>(a, B, s);
  if (tw == 8) return embed_dispatch<8>(a, B, s);
  if (tw == 16) return embed_dispatch<16>(a, B, s);
  return hipErrorInvalidValue;
}

hipError_t col_pass(const Tables& T, float2* work, int B, hipStream_t s) {
  PassArgs a = pass_args(T, work);
  a.table = T.propT;
  a.tw = T.twy;
  return pass_dispatch<PASS_COL>(T.ny, tw_of(T), T.nx, a, B, s, T.sched);
}

hipError_t col_gather(const Tables& T, float2* work, int B, void* basis, int D, const int32_t* wave_row, int split,
                      hipStream_t s) {
  PassArgs a = pass_args(T, work);
  a.table = T.propT;
  a.tw = T.twy;
  a.basis = basis;
  a.D = D;
  a.comp = T.compT;
  a.wave_row = wave_row;
  a.split_bf16 = split;
  return pass_dispatch<PASS_GATHER>(T.ny, tw_of(T), T.nx, a, B, s, T.sched);
}

hipError_t col_reduce(const Tables& T, float2* work, int B, const int32_t* wave_out, double* img, int ndet,
                      int64_t img_stride, double scale, hipStream_t s) {
  PassArgs a = pass_args(T, work);
  a.table = T.propT;
  a.tw = T.twy;
  a.mask = T.maskT;
  a.wave_row = wave_out;
  a.img = img;
  a.ndet = ndet;
  a.img_stride = img_stride;
  a.scale = scale;
  return pass_dispatch<PASS_REDUCE>(T.ny, tw_of(T), T.nx, a, B, s, T.sched);
}

static size_t contract_shm(const Contraction& c, int pt, int out) {
  return (size_t)pt * c.L * (sizeof(int64_t) + sizeof(float2)) +
         (out == OUT_RADIAL ? (size_t)pt * c.nbins * sizeof(double) : 0);
}

template <int SPLIT, int PT, int OUT>
static hipError_t contract_pt(const Contraction& c, int np, hipStream_t s) {
  dim3 grid((unsigned)c.nchunks, (unsigned)((np + PT - 1) / PT));
  k_contract<SPLIT, PT, OUT><<<grid, kCT, contract_shm(c, PT, OUT), s>>>(c);
  return hipGetLastError();
}

template <int OUT>
static hipError_t contract_out(const Contraction& c, int np, hipStream_t s) {
  // per-block tables of PT probes x L neighbours (and PT x nbins annulus sums) must fit
  // 64 KiB of LDS
  const bool wide = contract_shm(c, 8, OUT) <= 60 * 1024;
  if (!wide && contract_shm(c, 1, OUT) > 60 * 1024) return hipErrorInvalidValue;
  if (c.split_bf16) return wide ? contract_pt<1, 8, OUT>(c, np, s) : contract_pt<1, 1, OUT>(c, np, s);
  return wide ? contract_pt<0, 8, OUT>(c, np, s) : contract_pt<0, 1, OUT>(c, np, s);
}

hipError_t contract(const Contraction& c, hipStream_t s) {
  const int np = c.probe_list ? c.n_list : c.ww * c.wh;
  if (np <= 0 || c.nchunks <= 0) return hipSuccess;
  if (c.patterns) return contract_out<OUT_PATTERN>(c, np, s);
  if (c.radial) {
    if (!c.bin_of || c.nbins < 1 || c.nbins > kMaxRadialBins) return hipErrorInvalidValue;
    return contract_out<OUT_RADIAL>(c, np, s);
  }
  return contract_out<OUT_RINGS>(c, np, s);
}

__global__ void k_intensity(const float2* __restrict__ in, float* __restrict__ out, int64_t n, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 v = in[i];
  out[i] = (float)(scale * ((double)v.x * v.x + (double)v.y * v.y));
}

hipError_t intensity(const float2* in, float* out, int64_t n, double scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  k_intensity<<<(unsigned)((n + th - 1) / th), th, 0, s>>>(in, out, n, scale);
  return hipGetLastError();
}

// The same contraction with the K-steps of every sub-block split over two wavefronts (8 per
// workgroup): each holds half of the A fragments, the halves' complex sums meet in LDS before
// |psi|^2. Twice the wavefronts per workgroup fill the slab and hide each other's latency.
template <int SPLIT, int KH>
__global__ __launch_bounds__(512) void k_contract_mfma2(Stencil c) {
  extern __shared__ unsigned char dyn[];
  const int nt = c.W * c.H;
  float2* slab = reinterpret_cast<float2*>(dyn);                          // [nt][16]
  int32_t* rowid = reinterpret_cast<int32_t*>(slab + (size_t)nt * 16);    // [nt]
  __shared__ f32x4 part[4][2][64];                                        // upper halves' sums
  int ti, tj, chunk;
  stencil_item(c, ti, tj, chunk);
  const int ox = (c.ox0 + ti * c.tile_dx) % c.Rfx;
  const int oy = (c.oy0 + tj * c.tile_dy) % c.Rfy;
  for (int t = threadIdx.x; t < nt; t += 512) {
    const int x = t % c.W, y = t / c.W;
    rowid[t] = c.row_of[((oy + y) % c.Rfy) * c.Rfx + (ox + x) % c.Rfx];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sb = wv & 3, kh = wv >> 2;                  // sub-block, half of the K-steps
  const int kk = lane >> 4, n = lane & 15;
  const int k0 = kh * KH;
  float2 A[KH];
#pragma unroll
  for (int q = 0; q < KH; ++q) A[q] = k0 + q < c.nks ? c.a[(k0 + q) * 64 + lane] : make_float2(0.f, 0.f);
  const int base = (sb >> 1) * c.sub_dy * c.W + (sb & 1) * c.sub_dx + kk;
  const int start = c.chunk_start[chunk], len = c.chunk_len[chunk];
  const uint32_t mask = c.chunk_mask[chunk];
  double val[4] = {0.0, 0.0, 0.0, 0.0};
  for (int d0 = 0; d0 < len; d0 += 16) {
    __syncthreads();  // row ids written, previous slab and partial sums consumed
    const int rem = len - d0;
    constexpr int kFill = 4;
    for (int i0 = threadIdx.x; i0 < nt * 16; i0 += 512 * kFill) {
      float2 v[kFill];
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        const int i = i0 + u * 512;
        v[u] = make_float2(0.f, 0.f);
        if (i < nt * 16) {
          const int t = i >> 4, q = i & 15;
          const int r = rowid[t];
          if (r >= 0 && q < rem) v[u] = load_basis<SPLIT>(c.basis, (int64_t)r * c.D + start + d0 + q);
        }
      }
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        const int i = i0 + u * 512;
        if (i < nt * 16) slab[i] = v[u];
      }
    }
    __syncthreads();
    f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < KH; ++q) {
      if (k0 + q < c.nks) {
        const float2 b = slab[(base + c.ks_off[k0 + q]) * 16 + n];
        cre = __builtin_amdgcn_mfma_f32_16x16x4f32(A[q].x, b.x, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x4f32(A[q].x, b.y, cim, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-A[q].y, b.y, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x4f32(A[q].y, b.x, cim, 0, 0, 0);
      }
    }
    if (kh == 1) {
      part[sb][0][lane] = cre;
      part[sb][1][lane] = cim;
    }
    __syncthreads();
    if (kh == 0 && n < rem) {
      cre += part[sb][0][lane];
      cim += part[sb][1][lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) val[r] += (double)cre[r] * cre[r] + (double)cim[r] * cim[r];
    }
  }
  if (kh != 0) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double x = val[r];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o);
    val[r] = x;
  }
  if (n == 0) {
    const int by = tj * 8 + (sb >> 1) * 4 + kk;
    const int64_t stride = (int64_t)c.ww * c.wh;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int bx = ti * 8 + (sb & 1) * 4 + r;
      if (bx >= c.pa0 && bx < c.pa1 && by >= c.pb0 && by < c.pb1) {
        const double v = val[r] * c.scale;
        for (int d = 0; d < c.ndet; ++d)
          if (mask & (1u << d)) atomicAdd(c.img + (int64_t)d * stride + (int64_t)by * c.ww + bx, v);
      }
    }
  }
}

// The same with the slab copied from the basis straight into LDS (16 bytes per lane per
// instruction, no registers in between): every wavefront copies 8 translate rows of 16 pixels
// per instruction and all copies of a slab are in flight at once. FP32 basis only. Rows that
// are absent and pixels past the chunk copy 16 zero bytes; a pixel pair that straddles the
// chunk's end reads one value past it (inside the basis allocation, padded by 128 bytes),
// which lands in a column the epilogue ignores.
template <int KH>
__global__ __launch_bounds__(512) void k_contract_mfma2_dma(Stencil c) {
  extern __shared__ unsigned char dyn[];
  const int nt = c.W * c.H;
  const int ntp = (nt + 7) & ~7;                                          // whole 8-row copies
  float2* slab = reinterpret_cast<float2*>(dyn);                          // [ntp][16]
  int32_t* rowid = reinterpret_cast<int32_t*>(slab + (size_t)ntp * 16);   // [ntp]
  __shared__ f32x4 part[4][2][64];
  int ti, tj, chunk;
  stencil_item(c, ti, tj, chunk);
  const int ox = (c.ox0 + ti * c.tile_dx) % c.Rfx;
  const int oy = (c.oy0 + tj * c.tile_dy) % c.Rfy;
  for (int t = threadIdx.x; t < ntp; t += 512) {
    const int x = t % c.W, y = t / c.W;
    rowid[t] = t < nt ? c.row_of[((oy + y) % c.Rfy) * c.Rfx + (ox + x) % c.Rfx] : -1;
  }
  // the wavefront index as a uniform value: the tests of the K-steps' tail are scalar branches
  // (as per-lane branches, each K-step waited on a vector load of its offset before its LDS read)
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int sb = wv & 3, kh = wv >> 2;
  const int kk = lane >> 4, n = lane & 15;
  const int k0 = kh * KH;
  float2 A[KH];
#pragma unroll
  for (int q = 0; q < KH; ++q) A[q] = k0 + q < c.nks ? c.a[(k0 + q) * 64 + lane] : make_float2(0.f, 0.f);
  // the wavefront's K-step offsets, lane q holding step k0 + q (0 past the last step): each
  // step reads its offset from that lane into a scalar register
  static_assert(KH <= 64, "one offset per lane");
  const int koff = lane < KH && k0 + lane < c.nks ? c.ks_off[k0 + lane] : 0;
  const int base = (sb >> 1) * c.sub_dy * c.W + (sb & 1) * c.sub_dx + kk;
  const int start = c.chunk_start[chunk], len = c.chunk_len[chunk];
  const uint32_t mask = c.chunk_mask[chunk];
  const float2* basis = reinterpret_cast<const float2*>(c.basis);
  const int rr = lane >> 3, q0 = (lane & 7) * 2;       // row within the copy, first pixel of the pair
  double val[4] = {0.0, 0.0, 0.0, 0.0};
  for (int d0 = 0; d0 < len; d0 += 16) {
    __syncthreads();  // row ids written, previous slab and partial sums consumed
    const int rem = len - d0;
    for (int t0 = wv * 8; t0 < ntp; t0 += 64) {
      const int r = rowid[t0 + rr];
      const float2* src = (r >= 0 && q0 < rem) ? basis + (int64_t)r * c.D + start + d0 + q0 : c.zeros;
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(slab + (size_t)t0 * 16), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's copies are in LDS
    __syncthreads();
    f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
    // runs of four K-steps under one uniform test: a run's steps past the last one multiply
    // zero A fragments by the slab's first rows (finite values) and add exact zeros
#pragma unroll
    for (int qb = 0; qb < KH; qb += 4) {
      if (k0 + qb < c.nks) {
#pragma unroll
        for (int q = qb; q < qb + 4 && q < KH; ++q) {
          const float2 b = slab[(base + __builtin_amdgcn_readlane(koff, q)) * 16 + n];
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(A[q].x, b.x, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(A[q].x, b.y, cim, 0, 0, 0);
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-A[q].y, b.y, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(A[q].y, b.x, cim, 0, 0, 0);
        }
      }
    }
    if (kh == 1) {
      part[sb][0][lane] = cre;
      part[sb][1][lane] = cim;
    }
    __syncthreads();
    if (kh == 0 && n < rem) {
      cre += part[sb][0][lane];
      cim += part[sb][1][lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) val[r] += (double)cre[r] * cre[r] + (double)cim[r] * cim[r];
    }
  }
  if (kh != 0) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double x = val[r];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o);
    val[r] = x;
  }
  if (n == 0) {
    const int by = tj * 8 + (sb >> 1) * 4 + kk;
    const int64_t stride = (int64_t)c.ww * c.wh;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int bx = ti * 8 + (sb & 1) * 4 + r;
      if (bx >= c.pa0 && bx < c.pa1 && by >= c.pb0 && by < c.pb1) {
        const double v = val[r] * c.scale;
        for (int d = 0; d < c.ndet; ++d)
          if (mask & (1u << d)) atomicAdd(c.img + (int64_t)d * stride + (int64_t)by * c.ww + bx, v);
      }
    }
  }
}

// The contraction of a split-BF16 basis on the bf16 MFMA (v_mfma_f32_16x16x16_bf16, FP32
// accumulation). Basis values are stored as (hi, lo) bf16 pairs, x = hi + lo; the
// coefficients are split the same way on the host. A product of two split values keeps the
// three terms hi hi + hi lo + lo hi (the lo lo term is below 2^-16 of it), so each complex
// product takes 12 bf16 MFMAs: Re += Re A Re B - Im A Im B and Im += Re A Im B + Im A Re B, three
// terms each. One instruction covers 16 translates (4 K-steps): lane l holds, for lane group
// g = l / 16, the 4 translates of K-step 4 G + g at its pixel (B) and its probe's coefficients
// for them (A), so the slab rows are read 4 at a time. Slabs are the raw 8-byte split values,
// copied straight into LDS as for FP32.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
struct SplitA {
  bf16x4 rh, rl, ih, il;             // Re and Im of 4 coefficients, hi and lo parts
};

// the 4 bf16 at half `h` (0: low 16 bits, 1: high) of word w of 4 rows
__device__ __forceinline__ bf16x4 gather4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, int h) {
  uint2 r;
  if (h == 0) {
    r.x = (a & 0xFFFFu) | (b << 16);
    r.y = (c & 0xFFFFu) | (d << 16);
  } else {
    r.x = (a >> 16) | (b & 0xFFFF0000u);
    r.y = (c >> 16) | (d & 0xFFFF0000u);
  }
  return __builtin_bit_cast(bf16x4, r);
}

template <int GH>
__global__ __launch_bounds__(512) void k_contract_bf16(Stencil c) {
  extern __shared__ unsigned char dyn[];
  const int nt = c.W * c.H;
  const int ntp = (nt + 7) & ~7;
  float2* slab = reinterpret_cast<float2*>(dyn);                          // [ntp][16] raw split values
  int32_t* rowid = reinterpret_cast<int32_t*>(slab + (size_t)ntp * 16);   // [ntp]
  __shared__ f32x4 part[4][2][64];
  int ti, tj, chunk;
  stencil_item(c, ti, tj, chunk);
  const int ox = (c.ox0 + ti * c.tile_dx) % c.Rfx;
  const int oy = (c.oy0 + tj * c.tile_dy) % c.Rfy;
  for (int t = threadIdx.x; t < ntp; t += 512) {
    const int x = t % c.W, y = t / c.W;
    rowid[t] = t < nt ? c.row_of[((oy + y) % c.Rfy) * c.Rfx + (ox + x) % c.Rfx] : -1;
  }
  // uniform wavefront index (scalar tail test); each lane's LDS row of every K-step group is
  // formed once, before the slabs, instead of a vector load of its offset in every group
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int sb = wv & 3, kh = wv >> 2;
  const int g = lane >> 4, n = lane & 15, kk = lane >> 4;
  const int ng = (c.nks + 3) / 4;
  const int g0 = kh * GH;
  const SplitA* abf = reinterpret_cast<const SplitA*>(c.abf);
  SplitA A[GH];
#pragma unroll
  for (int q = 0; q < GH; ++q) {
    if (g0 + q < ng) {
      A[q] = abf[(g0 + q) * 64 + lane];
    } else {
      const bf16x4 z = {0, 0, 0, 0};
      A[q] = SplitA{z, z, z, z};
    }
  }
  const bf16x4 sign = {(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
  const int base0 = (sb >> 1) * c.sub_dy * c.W + (sb & 1) * c.sub_dx;
  int rowq[GH];
#pragma unroll
  for (int q = 0; q < GH; ++q) {
    const int ks = 4 * (g0 + q) + g;
    rowq[q] = base0 + (g0 + q < ng && ks < c.nks ? c.ks_off[ks] : 0);
  }
  const int start = c.chunk_start[chunk], len = c.chunk_len[chunk];
  const uint32_t mask = c.chunk_mask[chunk];
  const float2* basis = reinterpret_cast<const float2*>(c.basis);
  const int rr = lane >> 3, q0 = (lane & 7) * 2;
  double val[4] = {0.0, 0.0, 0.0, 0.0};
  for (int d0 = 0; d0 < len; d0 += 16) {
    __syncthreads();  // row ids written, previous slab and partial sums consumed
    const int rem = len - d0;
    for (int t0 = wv * 8; t0 < ntp; t0 += 64) {
      const int r = rowid[t0 + rr];
      const float2* src = (r >= 0 && q0 < rem) ? basis + (int64_t)r * c.D + start + d0 + q0 : c.zeros;
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(slab + (size_t)t0 * 16), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's copies are in LDS
    __syncthreads();
    f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
    const uint2* raw = reinterpret_cast<const uint2*>(slab);
#pragma unroll
    for (int q = 0; q < GH; ++q) {
      if (g0 + q < ng) {
        const int row = rowq[q];
        const uint2 r0 = raw[(row + 0) * 16 + n], r1 = raw[(row + 1) * 16 + n];
        const uint2 r2 = raw[(row + 2) * 16 + n], r3 = raw[(row + 3) * 16 + n];
        // word x: hi_re | lo_re << 16, word y: hi_im | lo_im << 16
        const bf16x4 brh = gather4(r0.x, r1.x, r2.x, r3.x, 0), brl = gather4(r0.x, r1.x, r2.x, r3.x, 1);
        const bf16x4 bih = gather4(r0.y, r1.y, r2.y, r3.y, 0), bil = gather4(r0.y, r1.y, r2.y, r3.y, 1);
        const SplitA& a = A[q];
        const bf16x4 nih = a.ih ^ sign, nil = a.il ^ sign;
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.rh, brh, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.rh, bih, cim, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.rh, brl, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.rh, bil, cim, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.rl, brh, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.rl, bih, cim, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nih, bih, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.ih, brh, cim, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nih, bil, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.ih, brl, cim, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nil, bih, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.il, brh, cim, 0, 0, 0);
      }
    }
    if (kh == 1) {
      part[sb][0][lane] = cre;
      part[sb][1][lane] = cim;
    }
    __syncthreads();
    if (kh == 0 && n < rem) {
      cre += part[sb][0][lane];
      cim += part[sb][1][lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) val[r] += (double)cre[r] * cre[r] + (double)cim[r] * cim[r];
    }
  }
  if (kh != 0) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double x = val[r];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o);
    val[r] = x;
  }
  if (n == 0) {
    const int by = tj * 8 + (sb >> 1) * 4 + kk;
    const int64_t stride = (int64_t)c.ww * c.wh;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int bx = ti * 8 + (sb & 1) * 4 + r;
      if (bx >= c.pa0 && bx < c.pa1 && by >= c.pb0 && by < c.pb1) {
        const double v = val[r] * c.scale;
        for (int d = 0; d < c.ndet; ++d)
          if (mask & (1u << d)) atomicAdd(c.img + (int64_t)d * stride + (int64_t)by * c.ww + bx, v);
      }
    }
  }
}

#ifndef LMA_CONTRACT_DMA
#define LMA_CONTRACT_DMA 1
#endif

template <int SPLIT, int KS>
static hipError_t stencil_ks(const Stencil& c, hipStream_t s) {
  const size_t shm = (size_t)c.W * c.H * (16 * sizeof(float2) + sizeof(int32_t));
  // split K over two wavefronts while each half keeps 4 wavefronts per SIMD (up to 80 K-steps)
  if constexpr (KS <= 80) {
    if (SPLIT && c.abf && c.zeros) {
      const int ntp = (c.W * c.H + 7) & ~7;
      const size_t shd = (size_t)ntp * (16 * sizeof(float2) + sizeof(int32_t));
      constexpr int GH = (KS / 2 + 3) / 4;   // 4-K-step groups per half
      const void* fb = reinterpret_cast<const void*>(&k_contract_bf16<GH>);
      hipError_t e = hipFuncSetAttribute(fb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shd);
      if (e != hipSuccess) return e;
      dim3 grid((unsigned)((int64_t)c.tiles_x * c.tiles_y * c.nchunks));
      k_contract_bf16<GH><<<grid, 512, shd, s>>>(c);
      return hipGetLastError();
    }
    if (LMA_CONTRACT_DMA && !SPLIT && c.zeros) {
      const int ntp = (c.W * c.H + 7) & ~7;
      const size_t shd = (size_t)ntp * (16 * sizeof(float2) + sizeof(int32_t));
      const void* fd = reinterpret_cast<const void*>(&k_contract_mfma2_dma<KS / 2>);
      hipError_t e = hipFuncSetAttribute(fd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shd);
      if (e != hipSuccess) return e;
      dim3 grid((unsigned)((int64_t)c.tiles_x * c.tiles_y * c.nchunks));
      k_contract_mfma2_dma<KS / 2><<<grid, 512, shd, s>>>(c);
      return hipGetLastError();
    }
    const void* fn = reinterpret_cast<const void*>(&k_contract_mfma2<SPLIT, KS / 2>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((int64_t)c.tiles_x * c.tiles_y * c.nchunks));
    k_contract_mfma2<SPLIT, KS / 2><<<grid, 512, shm, s>>>(c);
    return hipGetLastError();
  }
  const void* fn = reinterpret_cast<const void*>(&k_contract_mfma<SPLIT, KS>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((int64_t)c.tiles_x * c.tiles_y * c.nchunks));
  k_contract_mfma<SPLIT, KS><<<grid, 256, shm, s>>>(c);
  return hipGetLastError();
}

template <int SPLIT>
static hipError_t stencil_split(const Stencil& c, hipStream_t s) {
  if (c.nks <= 16) return stencil_ks<SPLIT, 16>(c, s);
  if (c.nks <= 32) return stencil_ks<SPLIT, 32>(c, s);
  if (c.nks <= 48) return stencil_ks<SPLIT, 48>(c, s);
  if (c.nks <= 64) return stencil_ks<SPLIT, 64>(c, s);
  if (c.nks <= 68) return stencil_ks<SPLIT, 68>(c, s);
  if (c.nks <= 80) return stencil_ks<SPLIT, 80>(c, s);
  return stencil_ks<SPLIT, 96>(c, s);
}

hipError_t contract_stencil(const Stencil& c, hipStream_t s) {
  if (c.tiles_x <= 0 || c.tiles_y <= 0 || c.nchunks <= 0) return hipSuccess;
  if (c.nks <= 0 || c.nks > kStencilMaxKs || c.W * c.H > kStencilMaxRect || c.W <= 0 || c.H <= 0)
    return hipErrorInvalidValue;
  return c.split_bf16 ? stencil_split<1>(c, s) : stencil_split<0>(c, s);
}

hipError_t fill_zero(double* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_zero<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n);
  return hipGetLastError();
}

hipError_t scale_out(double* out, const double* img, int64_t n, double w, int acc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_scale_out<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, img, n, w, acc);
  return hipGetLastError();
}

}  // namespace dev
}  // namespace lma

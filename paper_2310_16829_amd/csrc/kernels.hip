// gfx950 kernels of the LMA hot path.
//
// One multislice step (Fig. multislice_pseudocode) is two passes over the batch of waves:
//   row pass    : row IFFT (finishes the previous step's inverse transform), transmission
//                 exp(i sigma v_j), row FFT
//   column pass : column FFT, Fresnel propagator with band limit, column IFFT
// Between passes a wave lives in HBM in the mixed domain (x transformed, y spatial), so each
// step reads and writes every pixel twice: 32 bytes per pixel per slice per wave.
//
// Transforms are Stockham radix-8/4/2 FFTs with 8 elements per thread: N/8 threads per
// transform, each holding elements j + (N/8) m for m = 0..7 before every stage and after
// the last one, so consecutive transforms need no exchange; stages in between exchange
// through LDS. Twiddles come from FP64-computed tables rounded to FP32.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

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

template <int R, int DIR>
__device__ __forceinline__ void dft_r(float2* a) {
  if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 2) dft2<DIR>(a[0], a[1]);
}

// ------------------------------------------------------------------------------------------
// stage schedule: radix 8 while possible, the remaining factor (2 or 4) last
// ------------------------------------------------------------------------------------------
__host__ __device__ constexpr int fft_full8(int n) { int s = 0; while (n >= 8) { n /= 8; ++s; } return s; }
__host__ __device__ constexpr int fft_rest(int n) { while (n >= 8) n /= 8; return n; }
__host__ __device__ constexpr int fft_nstages(int n) { return fft_full8(n) + (fft_rest(n) > 1 ? 1 : 0); }
__host__ __device__ constexpr int fft_radix(int n, int s) { return s < fft_full8(n) ? 8 : fft_rest(n); }
__host__ __device__ constexpr int fft_span(int n, int s) {  // product of the radices before stage s
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fft_radix(n, i);
  return p;
}

// ------------------------------------------------------------------------------------------
// twiddles held in registers: for every stage after the first, the r-1 factors of each of
// the thread's 8/r butterflies
// ------------------------------------------------------------------------------------------
__host__ __device__ constexpr int tw_off(int n, int s) {
  int o = 0;
  for (int i = 1; i < s; ++i) o += 8 - 8 / fft_radix(n, i);
  return o;
}
__host__ __device__ constexpr int tw_count(int n) { return tw_off(n, fft_nstages(n)) > 0 ? tw_off(n, fft_nstages(n)) : 1; }

template <int N, int S>
__device__ __forceinline__ void tw_load_stage(float2* w, const float2* __restrict__ tab, int j) {
  constexpr int r = fft_radix(N, S), Ns = fft_span(N, S), Q = 8 / r, T = N / 8;
  constexpr int off = tw_off(N, S);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = (j + T * q) & (Ns - 1);
#pragma unroll
    for (int m = 1; m < r; ++m) w[off + q * (r - 1) + (m - 1)] = tab[m * k * (N / (Ns * r))];
  }
}

template <int N>
__device__ __forceinline__ void tw_load(float2* w, const float2* __restrict__ tab, int j) {
  constexpr int ns = fft_nstages(N);
  if constexpr (ns > 1) tw_load_stage<N, 1>(w, tab, j);
  if constexpr (ns > 2) tw_load_stage<N, (ns > 2 ? 2 : 1)>(w, tab, j);
  if constexpr (ns > 3) tw_load_stage<N, (ns > 3 ? 3 : 1)>(w, tab, j);
}

// One transform's exchange slot inside the pass tile: position p lives at p + p/2^PAD (one
// pad element every 2^PAD keeps the stride-8 Stockham writes on distinct banks of the
// 64 x 4-byte LDS).
#ifndef LMA_SLOT_PAD
#define LMA_SLOT_PAD 3
#endif
#ifndef LMA_TILE_EXTRA
#define LMA_TILE_EXTRA 3
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

template <int N, int DIR, int S, bool WL>
__device__ __forceinline__ void fft_stage(float2 (&v)[8], int j, const float2* w, const Slot& slot) {
  constexpr int r = fft_radix(N, S);
  constexpr int Ns = fft_span(N, S);
  constexpr int Q = 8 / r;
  constexpr int T = N / 8;
  constexpr bool last = (S == fft_nstages(N) - 1);
  constexpr int off = tw_off(N, S);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 a[r];
#pragma unroll
    for (int m = 0; m < r; ++m) a[m] = v[q + m * Q];
    const int b = j + T * q;
    const int k = b & (Ns - 1);
    if constexpr (Ns > 1) {
#pragma unroll
      for (int m = 1; m < r; ++m) a[m] = cmul(a[m], conj_if_inv<DIR>(w[off + q * (r - 1) + (m - 1)]));
    }
    dft_r<r, DIR>(a);
    if constexpr (last) {
#pragma unroll
      for (int m = 0; m < r; ++m) v[q + m * Q] = a[m];
    } else {
      const int base = (b / Ns) * Ns * r + k;
#pragma unroll
      for (int m = 0; m < r; ++m) slot.put(base + m * Ns, a[m]);
    }
  }
  if constexpr (!last) {
    exchange_sync<WL>();
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = slot.get(j + T * m);
    exchange_sync<WL>();
  }
}

// N-point transform of the 8 values held by thread j (of N/8); input and output at
// positions j + (N/8) m, natural order.
template <int N, int DIR, bool WL>
__device__ __forceinline__ void fft(float2 (&v)[8], int j, const float2* w, const Slot& slot) {
  constexpr int ns = fft_nstages(N);
  fft_stage<N, DIR, 0, WL>(v, j, w, slot);
  if constexpr (ns > 1) fft_stage<N, DIR, (ns > 1 ? 1 : 0), WL>(v, j, w, slot);
  if constexpr (ns > 2) fft_stage<N, DIR, (ns > 2 ? 2 : 0), WL>(v, j, w, slot);
  if constexpr (ns > 3) fft_stage<N, DIR, (ns > 3 ? 3 : 0), WL>(v, j, w, slot);
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
// Reads rows of length N from in[B][rows][N] (contiguous), transforms them, and stores the
// result transposed, out[B][N][rows], through an LDS tile of ROWS rows so that every store
// writes ROWS consecutive values. The row pass (rows = y, N = nx) takes the mixed domain
// [y][kx] to [kx][y]; the column pass (rows = kx, N = ny) takes [kx][y] back to [y][kx].
// Tables used by column passes are stored transposed, [kx][ky].
// ------------------------------------------------------------------------------------------
enum { PASS_ROW = 0, PASS_COL = 1, PASS_INIT = 2, PASS_GATHER = 3, PASS_REDUCE = 4 };

template <int N>
struct PassCfg {
  static constexpr int T = N / 8;                                   // threads per transform
  static constexpr bool WL = T <= 64;                               // transform inside one wavefront
  static constexpr int S = WL ? ((64 / T) < 16 ? 64 / T : 16) : 1;  // transforms per wavefront
  static constexpr int WPT = WL ? 1 : T / 64;                       // wavefronts per transform
  static constexpr int ROWS = N <= 512 ? 16 : (N == 1024 ? 8 : 4);  // tile rows
  // tile row stride: a padded slot plus LMA_TILE_EXTRA, chosen so that the 16 rows read at one
  // column by the transposed store fall on distinct banks
  static constexpr int RS = slot_pos(N - 1) + 1 + LMA_TILE_EXTRA;
  static constexpr int NTW = tw_count(N);
};

struct PassArgs {
  const float2* in;
  float2* out;
  int rows;                  // rows per batch entry
  const float2* table;       // ROW: t_j [rows][N]; COL/GATHER/REDUCE: P^T [rows][N]; INIT: spectrum^T
  const float2* tw;          // twiddles exp(-2 pi i t / N), t < N
  const int64_t* wave_u;     // INIT: [B][2] lattice units of each wave's position
  int64_t Qx, Qy;
  int nrow_freq;             // INIT: number of rows (kx) for the frequency index; N is ky
  void* basis;               // GATHER
  int D;
  const int32_t* comp;       // GATHER: detector pixel index [rows][N] or -1
  const int32_t* wave_row;   // GATHER: basis row per wave; REDUCE: image index per wave
  int split_bf16;
  const uint32_t* mask;      // REDUCE: ring bits [rows][N]
  double* img;
  int ndet;
  int64_t img_stride;
  double scale;
};

__device__ __forceinline__ void split_bf16(float x, __hip_bfloat16& hi, __hip_bfloat16& lo) {
  hi = __float2bfloat16(x);
  lo = __float2bfloat16(x - __bfloat162float(hi));
}

template <int N, int WAVES, int MODE>
__global__ __launch_bounds__(WAVES * 64) void k_pass(PassArgs a) {
  using C = PassCfg<N>;
  constexpr int T = C::T, S = C::S, ROWS = C::ROWS, RS = C::RS;
  constexpr int TPB = WAVES * S / C::WPT;                  // transforms in flight per block
  static_assert(TPB >= 1 && ROWS % TPB == 0, "tile rows must split evenly over the block");
  constexpr int RPW = ROWS / TPB;                          // rounds per block
  __shared__ float2 tile[(ROWS + 1) * RS];                 // last row: scratch of idle lanes
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int sub = C::WL ? lane / T : 0;                    // transform within the wavefront
  const int j = C::WL ? lane % T : tid % T;                // thread within the transform
  const int tslot = C::WL ? (tid >> 6) * S + sub : tid / T;  // transform slot within the block
  const bool active = !C::WL || sub < S;
  const int groups = a.rows / ROWS;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int B = gridDim.x / groups;
  const int grp = blk / B, w = blk % B;                    // an XCD owns a range of rows
  const int row0 = grp * ROWS;

  float2 tw[C::NTW];
  tw_load<N>(tw, a.tw, j);

  [[maybe_unused]] double acc[8];
  if constexpr (MODE == PASS_REDUCE) {
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.0;
  }

  // rows are prefetched one round ahead so that their loads overlap the current transforms
  [[maybe_unused]] float2 nxt[8];
  if constexpr (MODE != PASS_INIT) {
    const float2* src = a.in + ((size_t)w * a.rows + row0 + (active ? tslot : 0)) * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) nxt[m] = src[j + T * m];
  }

#pragma unroll 1
  for (int rr = 0; rr < RPW; ++rr) {
    const int r = rr * TPB + (active ? tslot : 0);         // tile row
    const int row = row0 + r;
    const Slot slot{tile + (active ? r : ROWS) * RS};
    float2 v[8];
    if constexpr (MODE == PASS_INIT) {
      // u(. - pos_w): spectrum times exp(-2 pi i (mx ux / Qx + my uy / Qy)), reduced exactly in
      // lattice units, phase in FP64; rows are kx, positions ky
      const int mx = freq_index(row, a.nrow_freq);
      const int64_t ux = a.wave_u[2 * w], uy = a.wave_u[2 * w + 1];
      const int64_t ax = (((int64_t)mx * ux) % a.Qx + a.Qx) % a.Qx;
      const float2* src = a.table + (size_t)row * N;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int ky = j + T * m;
        const int my = freq_index(ky, N);
        const int64_t ay = (((int64_t)my * uy) % a.Qy + a.Qy) % a.Qy;
        double sn, cs;
        sincospi(-2.0 * ((double)ax / (double)a.Qx + (double)ay / (double)a.Qy), &sn, &cs);
        v[m] = cmul(src[ky], make_float2((float)cs, (float)sn));
      }
      fft<N, +1, C::WL>(v, j, tw, slot);
    } else {
#pragma unroll
      for (int m = 0; m < 8; ++m) v[m] = nxt[m];
      if (rr + 1 < RPW) {
        const float2* src = a.in + ((size_t)w * a.rows + row + TPB) * N;
#pragma unroll
        for (int m = 0; m < 8; ++m) nxt[m] = src[j + T * m];
      }
      const float2* tab = a.table + (size_t)row * N;
      if constexpr (MODE == PASS_ROW) {
        fft<N, +1, C::WL>(v, j, tw, slot);
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = cmul(v[m], tab[j + T * m]);
        fft<N, -1, C::WL>(v, j, tw, slot);
      } else {
        fft<N, -1, C::WL>(v, j, tw, slot);
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = cmul(v[m], tab[j + T * m]);
        if constexpr (MODE == PASS_COL) {
          fft<N, +1, C::WL>(v, j, tw, slot);
        } else if constexpr (MODE == PASS_GATHER) {
          if (active) {
            const int64_t brow = a.wave_row[w];
            const int32_t* cm = a.comp + (size_t)row * N;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
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
            const uint32_t* mk = a.mask + (size_t)row * N;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
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
    if constexpr (MODE == PASS_ROW || MODE == PASS_COL || MODE == PASS_INIT) {
      if (active) {
#pragma unroll
        for (int m = 0; m < 8; ++m) slot.put(j + T * m, v[m]);
      }
    }
  }

  if constexpr (MODE == PASS_REDUCE) {
    // block reduction of the ring sums: wavefront shuffles, then LDS
    __syncthreads();
    double* part = reinterpret_cast<double*>(tile);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double x = acc[q];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
      if (lane == 0) part[(tid >> 6) * 8 + q] = x;
    }
    __syncthreads();
    if (tid < a.ndet) {
      double sum = 0.0;
      for (int i = 0; i < WAVES; ++i) sum += part[i * 8 + tid];
      atomicAdd(a.img + tid * a.img_stride + a.wave_row[w], sum * a.scale);
    }
  } else if constexpr (MODE != PASS_GATHER) {
    __syncthreads();
    // transposed store: out[w][x][row0 + r] for x < N, r < ROWS
    constexpr int NT = WAVES * 64;
    constexpr int XPER = NT / ROWS;
    const int tr = tid % ROWS, tx = tid / ROWS;
    float2* dst = a.out + (size_t)w * N * a.rows + row0 + tr;
#pragma unroll 4
    for (int x = tx; x < N; x += XPER) dst[(size_t)x * a.rows] = tile[tr * RS + slot_pos(x)];
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

template <int SPLIT, int kPT>
__global__ __launch_bounds__(kCT) void k_contract(Contraction c) {
  extern __shared__ unsigned char dyn[];
  int64_t* rows = reinterpret_cast<int64_t*>(dyn);                        // [kPT][L]
  float2* al = reinterpret_cast<float2*>(rows + (size_t)kPT * c.L);       // [kPT][L]
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

__global__ void k_scale_out(double* out, const double* img, int64_t n, double w, int acc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (acc ? out[i] : 0.0) + w * img[i];
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
bool supported(int nx, int ny) {
  auto ok = [](int n) { return n >= 16 && n <= 2048 && (n & (n - 1)) == 0; };
  return ok(nx) && ok(ny);
}

hipError_t transmission(const float* v, float2* t, int64_t n, double sigma, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  k_transmission<<<(unsigned)((n + th - 1) / th), th, 0, s>>>(v, t, n, sigma);
  return hipGetLastError();
}

// wavefronts per block of the slice pass (tunable; clamped to what the size allows)
static int g_pass_waves = 4;
void set_pass_waves(int w) { g_pass_waves = w; }

template <int N>
constexpr int max_waves() {
  using C = PassCfg<N>;
  return C::WL ? C::ROWS / C::S : C::WPT;
}

template <int N, int WAVES, int MODE>
static hipError_t pass_launch(const PassArgs& a, int B, hipStream_t s) {
  const int groups = a.rows / PassCfg<N>::ROWS;
  const unsigned grid = (unsigned)(B * groups);
  k_pass<N, WAVES, MODE><<<grid, WAVES * 64, 0, s>>>(a);
  return hipGetLastError();
}

template <int N, int MODE>
static hipError_t pass_waves(const PassArgs& a, int B, hipStream_t s) {
  if (a.rows % PassCfg<N>::ROWS) return hipErrorInvalidValue;
  constexpr int MW = max_waves<N>();
  if constexpr (!PassCfg<N>::WL) {
    return pass_launch<N, MW, MODE>(a, B, s);
  } else {
    int w = g_pass_waves;
    if (w > MW) w = MW;
    if constexpr (MW >= 16) { if (w >= 16) return pass_launch<N, 16, MODE>(a, B, s); }
    if constexpr (MW >= 8) { if (w >= 8) return pass_launch<N, 8, MODE>(a, B, s); }
    if constexpr (MW >= 4) { if (w >= 4) return pass_launch<N, 4, MODE>(a, B, s); }
    if constexpr (MW >= 2) { if (w >= 2) return pass_launch<N, 2, MODE>(a, B, s); }
    return pass_launch<N, 1, MODE>(a, B, s);
  }
}

template <int MODE>
static hipError_t pass_dispatch(int N, const PassArgs& a, int B, hipStream_t s) {
  switch (N) {
    case 16: return pass_waves<16, MODE>(a, B, s);
    case 32: return pass_waves<32, MODE>(a, B, s);
    case 64: return pass_waves<64, MODE>(a, B, s);
    case 128: return pass_waves<128, MODE>(a, B, s);
    case 256: return pass_waves<256, MODE>(a, B, s);
    case 512: return pass_waves<512, MODE>(a, B, s);
    case 1024: return pass_waves<1024, MODE>(a, B, s);
    case 2048: return pass_waves<2048, MODE>(a, B, s);
  }
  return hipErrorInvalidValue;
}

hipError_t init_waves(const Tables& T, float2* out, const int64_t* wave_u, int B, hipStream_t s) {
  PassArgs a{};
  a.out = out;
  a.rows = T.nx;
  a.table = T.specT;
  a.tw = T.twy;
  a.wave_u = wave_u;
  a.Qx = T.Qx;
  a.Qy = T.Qy;
  a.nrow_freq = T.nx;
  return pass_dispatch<PASS_INIT>(T.ny, a, B, s);
}

hipError_t row_pass(const Tables& T, const float2* in, float2* out, const float2* trans_j, int B, hipStream_t s) {
  PassArgs a{};
  a.in = in;
  a.out = out;
  a.rows = T.ny;
  a.table = trans_j;
  a.tw = T.twx;
  return pass_dispatch<PASS_ROW>(T.nx, a, B, s);
}

hipError_t col_pass(const Tables& T, const float2* in, float2* out, int B, hipStream_t s) {
  PassArgs a{};
  a.in = in;
  a.out = out;
  a.rows = T.nx;
  a.table = T.propT;
  a.tw = T.twy;
  return pass_dispatch<PASS_COL>(T.ny, a, B, s);
}

hipError_t col_gather(const Tables& T, const float2* in, int B, void* basis, int D, const int32_t* wave_row,
                      int split, hipStream_t s) {
  PassArgs a{};
  a.in = in;
  a.rows = T.nx;
  a.table = T.propT;
  a.tw = T.twy;
  a.basis = basis;
  a.D = D;
  a.comp = T.compT;
  a.wave_row = wave_row;
  a.split_bf16 = split;
  return pass_dispatch<PASS_GATHER>(T.ny, a, B, s);
}

hipError_t col_reduce(const Tables& T, const float2* in, int B, const int32_t* wave_out, double* img, int ndet,
                      int64_t img_stride, double scale, hipStream_t s) {
  PassArgs a{};
  a.in = in;
  a.rows = T.nx;
  a.table = T.propT;
  a.tw = T.twy;
  a.mask = T.maskT;
  a.wave_row = wave_out;
  a.img = img;
  a.ndet = ndet;
  a.img_stride = img_stride;
  a.scale = scale;
  return pass_dispatch<PASS_REDUCE>(T.ny, a, B, s);
}

template <int SPLIT, int PT>
static hipError_t contract_pt(const Contraction& c, int np, hipStream_t s) {
  dim3 grid((unsigned)c.nchunks, (unsigned)((np + PT - 1) / PT));
  const size_t shm = (size_t)PT * c.L * (sizeof(int64_t) + sizeof(float2));
  k_contract<SPLIT, PT><<<grid, kCT, shm, s>>>(c);
  return hipGetLastError();
}

hipError_t contract(const Contraction& c, hipStream_t s) {
  const int np = c.probe_list ? c.n_list : c.ww * c.wh;
  if (np <= 0 || c.nchunks <= 0) return hipSuccess;
  // per-block tables of PT probes x L neighbours must fit 64 KiB of LDS
  const bool wide = (size_t)8 * c.L * (sizeof(int64_t) + sizeof(float2)) <= 60 * 1024;
  if (c.split_bf16) return wide ? contract_pt<1, 8>(c, np, s) : contract_pt<1, 1>(c, np, s);
  return wide ? contract_pt<0, 8>(c, np, s) : contract_pt<0, 1>(c, np, s);
}

hipError_t scale_out(double* out, const double* img, int64_t n, double w, int acc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_scale_out<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, img, n, w, acc);
  return hipGetLastError();
}

}  // namespace dev
}  // namespace lma

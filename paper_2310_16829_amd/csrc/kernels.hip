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

// LDS exchange layouts. Row transforms: one padded row per transform. Column transforms:
// [position][column] so that a wavefront touches consecutive columns.
template <int N>
struct RowLds {
  float2* base;  // this transform's row
  __device__ __forceinline__ int idx(int p) const { return p + (p >> 3); }
  __device__ __forceinline__ void put(int p, float2 v) const { base[idx(p)] = v; }
  __device__ __forceinline__ float2 get(int p) const { return base[idx(p)]; }
  static constexpr int kSize = N + N / 8;
};
template <int C>
struct ColLds {
  float2* base;  // base + column
  __device__ __forceinline__ void put(int p, float2 v) const { base[p * C] = v; }
  __device__ __forceinline__ float2 get(int p) const { return base[p * C]; }
};

template <int N, int DIR, int S, class Lds>
__device__ __forceinline__ void fft_stage(float2 (&v)[8], int j, const float2* __restrict__ tw, const Lds& lds) {
  constexpr int r = fft_radix(N, S);
  constexpr int Ns = fft_span(N, S);
  constexpr int Q = 8 / r;
  constexpr int T = N / 8;
  constexpr bool last = (S == fft_nstages(N) - 1);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 a[r];
#pragma unroll
    for (int m = 0; m < r; ++m) a[m] = v[q + m * Q];
    const int b = j + T * q;
    const int k = b & (Ns - 1);
    if constexpr (Ns > 1) {
#pragma unroll
      for (int m = 1; m < r; ++m) a[m] = cmul(a[m], conj_if_inv<DIR>(tw[m * k * (N / (Ns * r))]));
    }
    dft_r<r, DIR>(a);
    if constexpr (last) {
#pragma unroll
      for (int m = 0; m < r; ++m) v[q + m * Q] = a[m];
    } else {
      const int base = (b / Ns) * Ns * r + k;
#pragma unroll
      for (int m = 0; m < r; ++m) lds.put(base + m * Ns, a[m]);
    }
  }
  if constexpr (!last) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = lds.get(j + T * m);
    __syncthreads();
  }
}

// N-point transform of the 8 values held by thread j (of N/8); input and output at
// positions j + (N/8) m, natural order.
template <int N, int DIR, class Lds>
__device__ __forceinline__ void fft(float2 (&v)[8], int j, const float2* __restrict__ tw, const Lds& lds) {
  constexpr int ns = fft_nstages(N);
  fft_stage<N, DIR, 0>(v, j, tw, lds);
  if constexpr (ns > 1) fft_stage<N, DIR, (ns > 1 ? 1 : 0)>(v, j, tw, lds);
  if constexpr (ns > 2) fft_stage<N, DIR, (ns > 2 ? 2 : 0)>(v, j, tw, lds);
  if constexpr (ns > 3) fft_stage<N, DIR, (ns > 3 ? 3 : 0)>(v, j, tw, lds);
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
// row pass
// ------------------------------------------------------------------------------------------
template <int NX>
struct RowCfg {
  static constexpr int T = NX / 8;
  static constexpr int Rmax = (256 / T) > 0 ? 256 / T : 1;
};

template <int NX, int R>
__global__ __launch_bounds__(R * (NX / 8)) void k_row_pass(float2* __restrict__ work, const float2* __restrict__ trans,
                                                          const float2* __restrict__ tw, int ny) {
  constexpr int T = NX / 8;
  __shared__ float2 sm[R * RowLds<NX>::kSize];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = threadIdx.x / T, j = threadIdx.x % T;
  // logical block = (row group, wave) with the wave fastest: an XCD owns a range of y
  const int B = gridDim.x / (ny / R);
  const int yg = blk / B, w = blk % B;
  const int y = yg * R + r;
  float2* row = work + ((size_t)w * ny + y) * NX;
  const float2* trow = trans + (size_t)y * NX;
  RowLds<NX> lds{sm + r * RowLds<NX>::kSize};
  float2 v[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) v[m] = row[j + T * m];
  fft<NX, +1>(v, j, tw, lds);
#pragma unroll
  for (int m = 0; m < 8; ++m) v[m] = cmul(v[m], trow[j + T * m]);
  fft<NX, -1>(v, j, tw, lds);
#pragma unroll
  for (int m = 0; m < 8; ++m) row[j + T * m] = v[m];
}

// ------------------------------------------------------------------------------------------
// column passes
// ------------------------------------------------------------------------------------------
enum { COL_INIT = 0, COL_MID = 1, COL_GATHER = 2, COL_REDUCE = 3 };

template <int NY>
struct ColCfg {
  static constexpr int C = NY <= 512 ? 16 : (NY == 1024 ? 8 : 4);
  static constexpr int T = NY / 8;
  static constexpr int kThreads = C * T;
};

struct ColArgs {
  float2* work;
  const float2* spec;      // INIT
  const float2* prop;      // MID / GATHER / REDUCE
  const float2* tw;
  const int64_t* wave_u;   // INIT: [B][2] lattice units
  int64_t Qx, Qy;
  void* basis;             // GATHER
  int D;
  const int32_t* comp_map;
  const int32_t* wave_row; // GATHER: basis row per wave; REDUCE: image index per wave
  int split_bf16;
  const uint32_t* detmask; // REDUCE
  double* img;
  int ndet;
  int64_t img_stride;
  double scale;
  int nx, ny;
};

__device__ __forceinline__ void split_bf16(float x, __hip_bfloat16& hi, __hip_bfloat16& lo) {
  hi = __float2bfloat16(x);
  lo = __float2bfloat16(x - __bfloat162float(hi));
}

template <int NY, int MODE>
__global__ __launch_bounds__(ColCfg<NY>::kThreads) void k_col_pass(ColArgs a) {
  constexpr int C = ColCfg<NY>::C;
  constexpr int T = ColCfg<NY>::T;
  __shared__ float2 sm[NY * C];
  const int nx = a.nx;
  const int tiles = nx / C;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int B = gridDim.x / tiles;
  const int tile = blk / B, w = blk % B;   // an XCD owns a range of columns
  const int c = threadIdx.x % C, j = threadIdx.x / C;
  const int col = tile * C + c;
  ColLds<C> lds{sm + c};
  float2* base = a.work + (size_t)w * NY * nx + col;
  float2 v[8];
  if constexpr (MODE == COL_INIT) {
    // u(. - pos_w): spectrum times exp(-2 pi i (mx ux / Qx + my uy / Qy)), exact in units
    const int mx = freq_index(col, nx);
    const int64_t ux = a.wave_u[2 * w], uy = a.wave_u[2 * w + 1];
    const int64_t ax = (((int64_t)mx * ux) % a.Qx + a.Qx) % a.Qx;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int ky = j + T * m;
      const int my = freq_index(ky, NY);
      const int64_t ay = (((int64_t)my * uy) % a.Qy + a.Qy) % a.Qy;
      double turns = (double)ax / (double)a.Qx + (double)ay / (double)a.Qy;
      double s, cc;
      sincospi(-2.0 * turns, &s, &cc);
      v[m] = cmul(a.spec[(size_t)ky * nx + col], make_float2((float)cc, (float)s));
    }
    fft<NY, +1>(v, j, a.tw, lds);
#pragma unroll
    for (int m = 0; m < 8; ++m) base[(size_t)(j + T * m) * nx] = v[m];
    return;
  } else {
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = base[(size_t)(j + T * m) * nx];
    fft<NY, -1>(v, j, a.tw, lds);
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = cmul(v[m], a.prop[(size_t)(j + T * m) * nx + col]);
    if constexpr (MODE == COL_MID) {
      fft<NY, +1>(v, j, a.tw, lds);
#pragma unroll
      for (int m = 0; m < 8; ++m) base[(size_t)(j + T * m) * nx] = v[m];
    } else if constexpr (MODE == COL_GATHER) {
      const int64_t row = a.wave_row[w];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int d = a.comp_map[(size_t)(j + T * m) * nx + col];
        if (d >= 0) {
          if (a.split_bf16) {
            __hip_bfloat16 q[4];
            split_bf16(v[m].x, q[0], q[1]);
            split_bf16(v[m].y, q[2], q[3]);
            reinterpret_cast<uint2*>(a.basis)[row * a.D + d] = *reinterpret_cast<uint2*>(q);
          } else {
            reinterpret_cast<float2*>(a.basis)[row * a.D + d] = v[m];
          }
        }
      }
    } else {  // COL_REDUCE
      double acc[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) acc[r] = 0.0;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const uint32_t mask = a.detmask[(size_t)(j + T * m) * nx + col];
        const double p = (double)v[m].x * v[m].x + (double)v[m].y * v[m].y;
#pragma unroll
        for (int r = 0; r < 8; ++r)
          if (mask & (1u << r)) acc[r] += p;
      }
      // block reduction: wavefront shuffles, then one partial per wavefront in LDS (the
      // exchange buffer is free: every thread has passed the last exchange's barrier)
      double* part = reinterpret_cast<double*>(sm);
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        double x = acc[r];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) part[wv * 8 + r] = x;
      }
      __syncthreads();
      if (threadIdx.x < a.ndet) {
        double s = 0.0;
        const int nw = (ColCfg<NY>::kThreads + 63) / 64;
        for (int i = 0; i < nw; ++i) s += part[i * 8 + threadIdx.x];
        atomicAdd(a.img + threadIdx.x * a.img_stride + a.wave_row[w], s * a.scale);
      }
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

template <int NX>
static hipError_t row_pass_n(const Tables& T, float2* work, const float2* trans_j, int B, hipStream_t s) {
  constexpr int R0 = RowCfg<NX>::Rmax;
  const int ny = T.ny;
  // R rows per block must divide ny
  if (ny % R0 == 0) {
    k_row_pass<NX, R0><<<(unsigned)(B * (ny / R0)), R0 * (NX / 8), 0, s>>>(work, trans_j, T.twx, ny);
  } else {
    k_row_pass<NX, 1><<<(unsigned)(B * ny), NX / 8, 0, s>>>(work, trans_j, T.twx, ny);
  }
  return hipGetLastError();
}

hipError_t row_pass(const Tables& T, float2* work, const float2* trans_j, int B, hipStream_t s) {
  switch (T.nx) {
    case 16: return row_pass_n<16>(T, work, trans_j, B, s);
    case 32: return row_pass_n<32>(T, work, trans_j, B, s);
    case 64: return row_pass_n<64>(T, work, trans_j, B, s);
    case 128: return row_pass_n<128>(T, work, trans_j, B, s);
    case 256: return row_pass_n<256>(T, work, trans_j, B, s);
    case 512: return row_pass_n<512>(T, work, trans_j, B, s);
    case 1024: return row_pass_n<1024>(T, work, trans_j, B, s);
    case 2048: return row_pass_n<2048>(T, work, trans_j, B, s);
  }
  return hipErrorInvalidValue;
}

template <int NY, int MODE>
static hipError_t col_launch(const ColArgs& a, int B, hipStream_t s) {
  constexpr int C = ColCfg<NY>::C;
  if (a.nx % C) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(B * (a.nx / C));
  k_col_pass<NY, MODE><<<grid, ColCfg<NY>::kThreads, 0, s>>>(a);
  return hipGetLastError();
}

template <int MODE>
static hipError_t col_dispatch(const ColArgs& a, int B, hipStream_t s) {
  switch (a.ny) {
    case 16: return col_launch<16, MODE>(a, B, s);
    case 32: return col_launch<32, MODE>(a, B, s);
    case 64: return col_launch<64, MODE>(a, B, s);
    case 128: return col_launch<128, MODE>(a, B, s);
    case 256: return col_launch<256, MODE>(a, B, s);
    case 512: return col_launch<512, MODE>(a, B, s);
    case 1024: return col_launch<1024, MODE>(a, B, s);
    case 2048: return col_launch<2048, MODE>(a, B, s);
  }
  return hipErrorInvalidValue;
}

static ColArgs base_args(const Tables& T, float2* work) {
  ColArgs a{};
  a.work = work;
  a.spec = T.spec_init;
  a.prop = T.prop;
  a.tw = T.twy;
  a.Qx = T.Qx;
  a.Qy = T.Qy;
  a.comp_map = T.comp_map;
  a.detmask = T.detmask;
  a.nx = T.nx;
  a.ny = T.ny;
  return a;
}

hipError_t init_waves(const Tables& T, float2* work, const int64_t* wave_u, int B, hipStream_t s) {
  ColArgs a = base_args(T, work);
  a.wave_u = wave_u;
  return col_dispatch<COL_INIT>(a, B, s);
}

hipError_t col_pass(const Tables& T, float2* work, int B, hipStream_t s) {
  return col_dispatch<COL_MID>(base_args(T, work), B, s);
}

hipError_t col_gather(const Tables& T, const float2* work, int B, void* basis, int D, const int32_t* wave_row,
                      int split, hipStream_t s) {
  ColArgs a = base_args(T, const_cast<float2*>(work));
  a.basis = basis;
  a.D = D;
  a.wave_row = wave_row;
  a.split_bf16 = split;
  return col_dispatch<COL_GATHER>(a, B, s);
}

hipError_t col_reduce(const Tables& T, const float2* work, int B, const int32_t* wave_out, double* img, int ndet,
                      int64_t img_stride, double scale, hipStream_t s) {
  ColArgs a = base_args(T, const_cast<float2*>(work));
  a.wave_row = wave_out;
  a.img = img;
  a.ndet = ndet;
  a.img_stride = img_stride;
  a.scale = scale;
  return col_dispatch<COL_REDUCE>(a, B, s);
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

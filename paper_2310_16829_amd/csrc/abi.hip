// extern "C" entry points of liblma.so: argument checks, device buffers of a plan, and the
// order of kernel launches for propagation, image formation and local recompute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lma.h"
#include "planner.hpp"

using lma::HostPlan;
using lma::cd;

namespace {

thread_local std::string g_last_error;

lma_status fail(lma_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

struct TimedLaunch {
  const char* name;
  hipEvent_t a, b;
};

struct KernelTotals {
  std::string name;
  int64_t launches = 0;
  double ms = 0.0;
};

}  // namespace

struct lma_plan {
  HostPlan h;
  bool host_only = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;           // created by lma_build_basis (LMA_OWN_STREAM)
  int device = 0;
  int B = 1;                         // waves per batch
  int tw = 0;                        // tile width of the wave layout
  int sched = -1;                    // radix schedule of the transforms (lma_tuning; -1: per length)
  bool basis_valid = false;
  // LMA_GRAPH: wave sequences by their buffers; a sequence seen twice is captured and replayed
  bool use_graph = false;
  struct Captured {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Captured> graphs;      // most recent last
  int n_captured = 0;
  int64_t dev_bytes = 0;
  std::vector<void*> allocs;

  // tables (those read by column passes transposed, [kx][ky])
  float2 *d_specT = nullptr, *d_propT = nullptr, *d_twx = nullptr, *d_twy = nullptr;
  float2* d_uspecT = nullptr;        // spectrum of the input wave u (the probe's unless another u)
  // option (ii): translate windows (window tables transposed like the cell's)
  float2 *d_wspecT = nullptr, *d_wpropT = nullptr, *d_wtwx = nullptr, *d_wtwy = nullptr;
  int64_t* d_zero_u = nullptr;       // [B][2] zeros: every window starts from the same wave
  float2* d_wwork = nullptr;         // [B][window tiles]
  int32_t* d_compT = nullptr;
  uint32_t* d_maskT = nullptr;
  int zc0 = 0, zc1 = 0;              // kx columns zero after every column pass (band gap)
  int wzc0 = 0, wzc1 = 0;            // the same on the translate windows
  int sc0 = 0, sc1 = 0;              // kx columns where the probe spectrum vanishes
  int uc0 = 0, uc1 = 0;              // ... and where the input wave u's spectrum does
  int pz34 = 0, wpz34 = 0;           // the propagator vanishes at ky in [3ny/8, 5ny/8) (cell, windows)
  int32_t *d_row_of = nullptr, *d_set_dx = nullptr, *d_set_dy = nullptr;
  int32_t *d_chunk_start = nullptr, *d_chunk_len = nullptr;
  uint32_t* d_chunk_mask = nullptr;
  float2* d_alpha = nullptr;
  lma::StencilPlan st;               // the window's contraction as a banded GEMM (if it applies)
  int32_t* d_ks_off = nullptr;
  float2* d_stencil_a = nullptr;
  uint16_t* d_stencil_abf = nullptr; // split-BF16 A fragments of the bf16 MFMA (split basis)
  // rectangle partition when the window's basis exceeds the residency budget
  bool partitioned = false;
  lma::PartPlan pp;
  int32_t* d_part_row_of = nullptr;  // [parts][Rfy*Rfx]
  int64_t* d_part_u = nullptr;       // fresh translate positions of every part, in part order
  int32_t* d_part_slot = nullptr;    // their resident rows
  int32_t* d_part_probes = nullptr;  // window probe indices of every part (per-pixel contraction)
  std::vector<int64_t> part_fresh_off, part_probe_off;
  int64_t* d_row_u = nullptr;        // [n_rows][2] translate positions in lattice units
  int32_t* d_row_id = nullptr;       // [n_rows] 0..n_rows-1
  int64_t* d_probe_u = nullptr;      // [n_probes][2]
  int32_t* d_probe_out = nullptr;    // [n_probes] image index
  // work
  void* d_basis = nullptr;           // [n_rows][D] x 8 bytes, + 128 bytes of padding
  float2* d_zeros = nullptr;         // 256 zero bytes
  float2* d_work = nullptr;          // [B][ny/TW][nx/TW][TW][TW] tiled waves
  float2* d_trans = nullptr;         // [cap][ny][nx]
  int trans_cap = 0;
  float* d_pot = nullptr;            // staging for host potentials
  int pot_cap = 0;
  double* d_img = nullptr;           // [ndet][n_probes]
  int32_t* d_bin_of = nullptr;       // 3-D output: annulus of each detector pixel
  double bin_width = 0.0;
  int bin_count = 0;
  int32_t* d_list = nullptr;         // scratch index list (recompute)
  int64_t* d_list_u = nullptr;
  int list_cap = 0;

  // timing
  bool timing = false;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<KernelTotals> totals;
};

namespace {

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LMA_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

lma_status dalloc(lma_plan* p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(LMA_ERR_OOM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed: " +
                                 hipGetErrorString(e));
  }
  p->allocs.push_back(*ptr);
  p->dev_bytes += (int64_t)bytes;
  return LMA_OK;
}

template <class T>
lma_status upload(lma_plan* p, T** dst, const T* src, size_t n) {
  lma_status s = dalloc(p, reinterpret_cast<void**>(dst), n * sizeof(T));
  if (s != LMA_OK) return s;
  if (n) HIP_TRY(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
  return LMA_OK;
}

void free_one(lma_plan* p, void* ptr, size_t bytes) {
  if (!ptr) return;
  auto it = std::find(p->allocs.begin(), p->allocs.end(), ptr);
  if (it != p->allocs.end()) p->allocs.erase(it);
  (void)hipFree(ptr);
  p->dev_bytes -= (int64_t)bytes;
}

// The band gap of a transposed propagator table propT [nx][ny] (as uploaded): the longest run
// of kx columns where it is exactly zero for every ky and no detector pixel lies (compT, if
// given); a column pass leaves exact zeros there.
void band_gap(const std::vector<float2>& propT, int nx, int ny, const int32_t* compT, int* c0, int* c1) {
  auto zero_col = [&](int c) {
    for (int y = 0; y < ny; ++y) {
      const float2 q = propT[(size_t)c * ny + y];
      if (q.x != 0.f || q.y != 0.f || (compT && compT[(size_t)c * ny + y] >= 0)) return false;
    }
    return true;
  };
  int best0 = 0, best1 = 0;
  for (int x = 0; x < nx;) {
    if (!zero_col(x)) { ++x; continue; }
    int e = x;
    while (e < nx && zero_col(e)) ++e;
    if (e - x > best1 - best0) { best0 = x; best1 = e; }
    x = e;
  }
  *c0 = best0;
  *c1 = best1;
}

// The kx-column gaps of a plan from its tables as the device holds them (FP32, transposed):
// the band gap of the propagator (no detector pixel inside), the gaps of the probe spectrum and
// of u's, and the band gap of the translate windows' propagator.
void compute_gaps(lma_plan* p) {
  const HostPlan& h = p->h;
  const int nx = h.op.nx, ny = h.op.ny;
  const double XY = (double)nx * ny;
  auto f2T = [](const std::vector<cd>& src, int w, int hh, double scale) {
    std::vector<float2> t((size_t)w * hh);
    for (int y = 0; y < hh; ++y)
      for (int x = 0; x < w; ++x) {
        const cd& z = src[(size_t)y * w + x];
        t[(size_t)x * hh + y] = make_float2((float)(z.real() * scale), (float)(z.imag() * scale));
      }
    return t;
  };
  std::vector<int32_t> compT((size_t)nx * ny);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) compT[(size_t)x * ny + y] = h.comp_map[(size_t)y * nx + x];
  band_gap(f2T(h.prop, nx, ny, 1.0), nx, ny, compT.data(), &p->zc0, &p->zc1);
  band_gap(f2T(h.spec, nx, ny, 1.0 / XY), nx, ny, nullptr, &p->sc0, &p->sc1);
  if (h.lat.basis_kind == LMA_BASIS_PROBE) {
    p->uc0 = p->sc0;
    p->uc1 = p->sc1;
  } else {
    band_gap(f2T(h.uspec, nx, ny, 1.0 / XY), nx, ny, nullptr, &p->uc0, &p->uc1);
  }
  if (h.wnx > 0) band_gap(f2T(h.wprop, h.wnx, h.wny, 1.0), h.wnx, h.wny, nullptr, &p->wzc0, &p->wzc1);
  // ky positions [3n/8, 5n/8) where the propagator (as uploaded, FP32) is zero for every kx
  auto zero34 = [](const std::vector<cd>& prop, int w, int hh) {
    for (int y = 3 * hh / 8; y < 5 * hh / 8; ++y)
      for (int x = 0; x < w; ++x) {
        const cd& z = prop[(size_t)y * w + x];
        if ((float)z.real() != 0.f || (float)z.imag() != 0.f) return 0;
      }
    return 1;
  };
  p->pz34 = zero34(h.prop, nx, ny);
  if (h.wnx > 0) p->wpz34 = zero34(h.wprop, h.wnx, h.wny);
}

lma::dev::Tables window_tables(const lma_plan* p) {
  lma::dev::Tables t;
  t.nx = p->h.wnx;
  t.ny = p->h.wny;
  t.tw = lma::dev::tile_width(p->h.wnx, p->h.wny);
  t.Qx = p->h.Qx;
  t.Qy = p->h.Qy;
  t.specT = p->d_wspecT;
  t.propT = p->d_wpropT;
  t.twx = p->d_wtwx;
  t.twy = p->d_wtwy;
  t.zc0 = p->wzc0;
  t.zc1 = p->wzc1;
  t.prop_z34 = p->wpz34;
  return t;
}

lma::dev::Tables tables(const lma_plan* p) {
  lma::dev::Tables t;
  t.nx = p->h.op.nx;
  t.ny = p->h.op.ny;
  t.tw = p->tw;
  t.Qx = p->h.Qx;
  t.Qy = p->h.Qy;
  t.specT = p->d_specT;
  t.propT = p->d_propT;
  t.twx = p->d_twx;
  t.twy = p->d_twy;
  t.compT = p->d_compT;
  t.maskT = p->d_maskT;
  t.zc0 = p->zc0;
  t.zc1 = p->zc1;
  t.prop_z34 = p->pz34;
  t.sched = p->sched;
  return t;
}

std::vector<float2> twiddles(int n) {
  std::vector<float2> w(n);
  const double pi = 3.14159265358979323846;
  for (int t = 0; t < n; ++t) {
    double a = -2.0 * pi * (double)t / (double)n;
    w[t] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return w;
}

// bf16 of a float, rounded to nearest even (the device's conversion), and back
uint16_t bf16_round(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int64_t wave_bytes(const lma_optics& op) { return (int64_t)op.nx * op.ny * (int64_t)sizeof(float2); }

int auto_batch(const HostPlan& h) {
  if (h.lat.batch > 0) return h.lat.batch;
  // 2 GiB of waves, but at least 256 waves while they fit 4 GiB, at most 4096 (measured at the
  // medium workload, 512^2 with its band gap: 1024-wave batches 2.5 % faster per step than 512
  // and as fast as 2048, 64-256 waves 5-25 % slower; at 1024^2, 256 waves ran 9 % faster per
  // wave than 128, and at 2048^2 128 waves 4 % faster than 32)
  const int64_t wb = wave_bytes(h.op);
  int64_t b = std::max(((int64_t)2 << 30) / wb, std::min<int64_t>(256, ((int64_t)4 << 30) / wb));
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

// launch bookkeeping for kernel timing. A plan that times its launches holds a fixed pool of
// kTimingEvents events, created by lma_set_timing; each launch records a pair. When the pool
// runs dry, the recorded pairs are read out (the stream is synchronised) and their events
// return to the pool, so the live events stay bounded however many launches a call makes (a
// medium-workload propagation makes about 6,500).
constexpr size_t kTimingEvents = 256;

void collect_timing(lma_plan* p) {
  if (p->pending.empty()) return;
  (void)hipStreamSynchronize(p->stream);
  for (auto& t : p->pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    auto it = std::find_if(p->totals.begin(), p->totals.end(), [&](const KernelTotals& k) { return k.name == t.name; });
    if (it == p->totals.end()) {
      p->totals.push_back({t.name, 0, 0.0});
      it = p->totals.end() - 1;
    }
    it->launches += 1;
    it->ms += ms;
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  p->pending.clear();
}

struct Launch {
  lma_plan* p;
  const char* name;
  hipEvent_t a = nullptr;
  Launch(lma_plan* plan, const char* n) : p(plan), name(n) {
    if (!p->timing) return;
    a = take_event(p);
    if (a && hipEventRecord(a, p->stream) != hipSuccess) {
      p->event_pool.push_back(a);
      a = nullptr;
    }
  }
  static hipEvent_t take_event(lma_plan* p) {
    if (p->event_pool.empty()) collect_timing(p);
    if (p->event_pool.empty()) return nullptr;
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  void done() {
    if (!a) return;   // timing off, or this launch is not timed
    hipEvent_t b = take_event(p);
    if (!b || hipEventRecord(b, p->stream) != hipSuccess) {
      if (b) p->event_pool.push_back(b);
      p->event_pool.push_back(a);
      return;
    }
    p->pending.push_back({name, a, b});
  }
};

#define LAUNCH(plan, name, call)                                                          \
  do {                                                                                    \
    Launch l_(plan, name);                                                                \
    hipError_t e_ = (call);                                                               \
    l_.done();                                                                            \
    if (e_ != hipSuccess) return fail(LMA_ERR_DEVICE, std::string(name) + ": " + hipGetErrorString(e_)); \
  } while (0)

// room for nslices transmission tables
lma_status ensure_trans(lma_plan* p, int nslices) {
  const int64_t XY = (int64_t)p->h.op.nx * p->h.op.ny;
  if (nslices > p->trans_cap) {
    free_one(p, p->d_trans, (size_t)p->trans_cap * XY * sizeof(float2));
    p->d_trans = nullptr;
    p->trans_cap = 0;
    lma_status s = dalloc(p, reinterpret_cast<void**>(&p->d_trans), (size_t)nslices * XY * sizeof(float2));
    if (s != LMA_OK) return s;
    p->trans_cap = nslices;
  }
  return LMA_OK;
}

// transmission tables t_j = exp(i sigma v_j) for the given potential
lma_status prepare_transmission(lma_plan* p, const float* potential, int nslices, int32_t flags) {
  const int64_t XY = (int64_t)p->h.op.nx * p->h.op.ny;
  if (lma_status s = ensure_trans(p, nslices); s != LMA_OK) return s;
  const float* src = potential;
  if (!(flags & LMA_PTR_DEVICE)) {
    if (nslices > p->pot_cap) {
      free_one(p, p->d_pot, (size_t)p->pot_cap * XY * sizeof(float));
      p->d_pot = nullptr;
      p->pot_cap = 0;
      lma_status s = dalloc(p, reinterpret_cast<void**>(&p->d_pot), (size_t)nslices * XY * sizeof(float));
      if (s != LMA_OK) return s;
      p->pot_cap = nslices;
    }
    HIP_TRY(hipMemcpyAsync(p->d_pot, potential, (size_t)nslices * XY * sizeof(float), hipMemcpyHostToDevice, p->stream));
    src = p->d_pot;
  }
  LAUNCH(p, "transmission", lma::dev::transmission(src, p->d_trans, (int64_t)nslices * XY, p->h.op.sigma, p->stream));
  return LMA_OK;
}

// Buffers a slice loop works in: the wave batch (B waves, tiled), the transmission tables and
// the image accumulator. The plan's own, or caller-provided ones of the same layout.
struct WaveBufs {
  float2* work;
  const float2* trans;
  double* img;
  int B;
};
WaveBufs plan_bufs(const lma_plan* p) { return {p->d_work, p->d_trans, p->d_img, p->B}; }

// multislice of waves [first, first + n) of a position list; the last column pass either
// gathers the detector pixels into rows of `target` (wave_row != null; the resident basis
// unless given) or reduces into the image (wave_out != null). Probe waves (no wave_row) start
// from psi_0, translates from u.
lma_status run_waves(lma_plan* p, const int64_t* d_u, const int32_t* d_row, const int32_t* d_out, int n, int nslices,
                     void* target = nullptr, bool probes = false, const WaveBufs* wb = nullptr) {
  const WaveBufs bf = wb ? *wb : plan_bufs(p);
  const lma::dev::Tables T = tables(p);
  const int64_t XY = (int64_t)p->h.op.nx * p->h.op.ny;
  const int split = target ? 0 : p->h.lat.precision == LMA_GEMM_SPLIT_BF16;
  if (p->h.wnx > 0 && d_row && !probes) {
    // option (ii): translates on windows centred on them, the last step on the cell
    if (bf.B > p->B) return fail(LMA_ERR_ARG, "wave batch larger than the window buffer");
    const lma::dev::Tables Tw = window_tables(p);
    for (int first = 0; first < n; first += bf.B) {
      const int nb = std::min(bf.B, n - first);
      const int64_t* u = d_u + 2 * (int64_t)first;
      LAUNCH(p, "init", lma::dev::init_waves(Tw, p->d_wwork, p->d_zero_u, nb, p->stream));
      for (int j = 0; j < nslices; ++j) {
        const bool last = j + 1 == nslices;
        LAUNCH(p, "row_pass", lma::dev::row_pass_window(Tw, p->d_wwork, bf.trans + (size_t)j * XY, T.nx, T.ny, u,
                                                        T.Qx, T.Qy, last, j > 0, nb, p->stream));
        if (!last) LAUNCH(p, "col_pass", lma::dev::col_pass(Tw, p->d_wwork, nb, p->stream));
      }
      LAUNCH(p, "embed", lma::dev::embed_windows(T, bf.work, Tw, p->d_wwork, u, nb, p->stream));
      LAUNCH(p, "col_gather", lma::dev::col_gather(T, bf.work, nb, target ? target : p->d_basis, p->h.D(),
                                                   d_row + first, split, p->stream));
    }
    return LMA_OK;
  }
  // translates start from u, probes from psi_0; the initial waves skip, and the first row
  // pass does not read, the kx columns where that spectrum vanishes
  lma::dev::Tables Ti = T;
  const bool from_u = d_row && !probes;
  if (from_u) Ti.specT = p->d_uspecT;
  Ti.ic0 = from_u ? p->uc0 : p->sc0;
  Ti.ic1 = from_u ? p->uc1 : p->sc1;
  for (int first = 0; first < n; first += bf.B) {
    const int nb = std::min(bf.B, n - first);
    LAUNCH(p, "init", lma::dev::init_waves(Ti, bf.work, d_u + 2 * (int64_t)first, nb, p->stream));
    for (int j = 0; j < nslices; ++j) {
      LAUNCH(p, "row_pass", lma::dev::row_pass(Ti, bf.work, bf.trans + (size_t)j * XY, nb, j > 0, p->stream));
      if (j + 1 < nslices) {
        LAUNCH(p, "col_pass", lma::dev::col_pass(T, bf.work, nb, p->stream));
      } else if (d_row) {
        LAUNCH(p, "col_gather", lma::dev::col_gather(T, bf.work, nb, target ? target : p->d_basis, p->h.D(), d_row + first,
                                                     split, p->stream));
      } else {
        LAUNCH(p, "col_reduce", lma::dev::col_reduce(T, bf.work, nb, d_out + first, bf.img, p->h.ndet,
                                                     p->h.n_probes(), (double)XY, p->stream));
      }
    }
  }
  return LMA_OK;
}

// run_waves through a HIP graph (LMA_GRAPH): the first call of a sequence runs eagerly and
// records its key (every buffer and size its kernels take); the second captures it and
// every later one replays the graph. Graphs hold kernel launches only.
constexpr size_t kMaxGraphs = 8;
lma_status waves(lma_plan* p, const int64_t* d_u, const int32_t* d_row, const int32_t* d_out, int n, int nslices) {
  if (!p->use_graph || p->timing || !p->stream) return run_waves(p, d_u, d_row, d_out, n, nslices);
  std::vector<int64_t> key = {(int64_t)(intptr_t)d_u, (int64_t)(intptr_t)d_row, (int64_t)(intptr_t)d_out, n, nslices,
                              (int64_t)(intptr_t)p->d_trans, (int64_t)(intptr_t)p->d_work,
                              (int64_t)(intptr_t)p->d_basis, (int64_t)(intptr_t)p->d_img, p->B};
  auto it = std::find_if(p->graphs.begin(), p->graphs.end(), [&](const lma_plan::Captured& c) { return c.key == key; });
  if (it == p->graphs.end()) {
    if (p->graphs.size() >= kMaxGraphs) {
      if (p->graphs.front().exec) (void)hipGraphExecDestroy(p->graphs.front().exec);
      p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back({key, nullptr});
    return run_waves(p, d_u, d_row, d_out, n, nslices);
  }
  if (!it->exec) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed));
    lma_status s = run_waves(p, d_u, d_row, d_out, n, nslices);
    hipError_t e = hipStreamEndCapture(p->stream, &g);
    if (s != LMA_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it->exec = x;
    ++p->n_captured;
  }
  HIP_TRY(hipGraphLaunch(it->exec, p->stream));
  return LMA_OK;
}

lma_status ensure_list(lma_plan* p, int n) {
  if (n <= p->list_cap) return LMA_OK;
  free_one(p, p->d_list, (size_t)p->list_cap * sizeof(int32_t));
  free_one(p, p->d_list_u, (size_t)p->list_cap * 2 * sizeof(int64_t));
  p->d_list = nullptr;
  p->d_list_u = nullptr;
  p->list_cap = 0;
  lma_status s = dalloc(p, reinterpret_cast<void**>(&p->d_list), (size_t)n * sizeof(int32_t));
  if (s != LMA_OK) return s;
  s = dalloc(p, reinterpret_cast<void**>(&p->d_list_u), (size_t)n * 2 * sizeof(int64_t));
  if (s != LMA_OK) return s;
  p->list_cap = n;
  return LMA_OK;
}

lma::dev::Contraction contraction(const lma_plan* p) {
  const HostPlan& h = p->h;
  lma::dev::Contraction c;
  c.basis = p->d_basis;
  c.split_bf16 = h.lat.precision == LMA_GEMM_SPLIT_BF16;
  c.D = h.D();
  c.row_of = p->d_row_of;
  c.set_dx = p->d_set_dx;
  c.set_dy = p->d_set_dy;
  c.alpha = p->d_alpha;
  c.L = h.lat.L;
  c.Rfx = h.Rfx;
  c.Rfy = h.Rfy;
  c.ncls_x = h.ncls_x;
  c.ncls_y = h.ncls_y;
  c.stepx = h.Rfx / h.gx;
  c.stepy = h.Rfy / h.gy;
  c.wa0 = h.wa0;
  c.wb0 = h.wb0;
  c.ww = h.ww;
  c.wh = h.wh;
  c.chunk_start = p->d_chunk_start;
  c.chunk_len = p->d_chunk_len;
  c.chunk_mask = p->d_chunk_mask;
  c.nchunks = (int)h.chunk_start.size();
  c.ndet = h.ndet;
  c.scale = (double)h.op.nx * h.op.ny;
  c.img = p->d_img;
  return c;
}

lma::dev::Stencil stencil(const lma_plan* p) {
  const HostPlan& h = p->h;
  const lma::StencilPlan& st = p->st;
  lma::dev::Stencil c;
  c.basis = p->d_basis;
  c.split_bf16 = h.lat.precision == LMA_GEMM_SPLIT_BF16;
  c.D = h.D();
  c.row_of = p->d_row_of;
  c.Rfx = h.Rfx;
  c.Rfy = h.Rfy;
  c.nks = st.nks;
  c.W = st.W;
  c.H = st.H;
  c.ox0 = st.ox0;
  c.oy0 = st.oy0;
  c.tile_dx = st.tile_dx;
  c.tile_dy = st.tile_dy;
  c.sub_dx = st.sub_dx;
  c.sub_dy = st.sub_dy;
  c.tiles_x = st.tiles_x;
  c.tiles_y = st.tiles_y;
  c.tile_x0 = 0;
  c.tile_y0 = 0;
  c.ks_off = p->d_ks_off;
  c.a = p->d_stencil_a;
  c.abf = p->d_stencil_abf;
  c.ww = h.ww;
  c.wh = h.wh;
  c.pa0 = 0;
  c.pa1 = h.ww;
  c.pb0 = 0;
  c.pb1 = h.wh;
  c.chunk_start = p->d_chunk_start;
  c.chunk_len = p->d_chunk_len;
  c.chunk_mask = p->d_chunk_mask;
  c.nchunks = (int)h.chunk_start.size();
  c.ndet = h.ndet;
  c.scale = (double)h.op.nx * h.op.ny;
  c.img = p->d_img;
  c.zeros = p->d_zeros;
  return c;
}

lma_status write_image(lma_plan* p, double* image, int32_t flags, double weight) {
  const int64_t n = (int64_t)p->h.ndet * p->h.n_probes();
  if (flags & LMA_PTR_DEVICE) {
    LAUNCH(p, "scale_out", lma::dev::scale_out(image, p->d_img, n, weight, (flags & LMA_ACCUMULATE) ? 1 : 0, p->stream));
    return LMA_OK;
  }
  std::vector<double> tmp((size_t)n);
  HIP_TRY(hipMemcpyAsync(tmp.data(), p->d_img, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (flags & LMA_ACCUMULATE)
    for (int64_t i = 0; i < n; ++i) image[i] += weight * tmp[i];
  else
    for (int64_t i = 0; i < n; ++i) image[i] = weight * tmp[i];
  return LMA_OK;
}

int64_t footprint_of(const HostPlan& h, int B, int nslices, bool with_basis) {
  const int64_t XY = (int64_t)h.op.nx * h.op.ny;
  int64_t b = 0;
  b += XY * (8 + 8 + 4 + 4);                          // spectrum, propagator, compaction map, ring masks
  b += (int64_t)(h.op.nx + h.op.ny) * 8;              // twiddles
  b += h.n_translates() * 4;                          // row map
  b += (int64_t)h.nsets * h.lat.L * (4 + 4 + 8);      // neighbours, coefficients
  b += (int64_t)h.chunk_start.size() * 12;
  b += (int64_t)h.rows.size() * 20 + h.n_probes() * 20;
  b += (int64_t)h.ndet * h.n_probes() * 8;            // image
  b += (int64_t)B * XY * 8;                           // wave batch
  b += (int64_t)nslices * XY * (8 + 4);               // transmission tables and potential staging
  if (with_basis) b += (int64_t)h.rows.size() * h.D() * 8 + 128;
  b += 256;                                           // zero bytes
  if (h.wnx > 0) b += (int64_t)h.wnx * h.wny * (8 + 8) + (int64_t)B * (h.wnx * h.wny * 8 + 16);   // window tables, batch
  return b;
}

}  // namespace

// ==============================================================================================
// extern "C"
// ==============================================================================================
namespace lma {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace lma

extern "C" {

const char* lma_last_error(void) { return g_last_error.c_str(); }

lma_status lma_electron_constants(double kv, double* wavelength, double* sigma) {
  if (!(kv > 0) || !std::isfinite(kv)) return fail(LMA_ERR_ARG, "kv must be positive");
  lma::electron_constants(kv, wavelength, sigma);
  return LMA_OK;
}

lma_status lma_footprint(const lma_optics* optics, const lma_lattice* lattice, const lma_detectors* detectors,
                         int32_t nslices, int64_t* bytes) {
  if (!bytes) return fail(LMA_ERR_ARG, "bytes is null");
  if (nslices < 1) return fail(LMA_ERR_ARG, "nslices must be >= 1");
  try {
    HostPlan h;
    std::string err;
    lma_status s = lma::build_host_plan(optics, lattice, detectors, &h, &err);
    if (s != LMA_OK) return fail(s, err);
    int B = auto_batch(h);
    B = (int)std::min<int64_t>(B, std::max<int64_t>(std::max<int64_t>((int64_t)h.rows.size(), h.n_probes()), 1));
    *bytes = footprint_of(h, B, nslices, true);
    return LMA_OK;
  } catch (const std::bad_alloc&) {
    return fail(LMA_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(LMA_ERR_ARG, e.what());
  }
}

static void release(lma_plan* p) {
  if (!p) return;
  for (auto& t : p->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : p->event_pool) (void)hipEventDestroy(e);
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

void lma_destroy(lma_plan* plan) {
  if (!plan) return;
  if (!plan->host_only) (void)hipStreamSynchronize(plan->stream);
  release(plan);
}

lma_status lma_build_basis(const lma_optics* optics, const lma_lattice* lattice, const lma_detectors* detectors,
                           void* hip_stream, int32_t flags, lma_plan** out) {
  if (!out) return fail(LMA_ERR_ARG, "out is null");
  *out = nullptr;
  lma_plan* p = nullptr;
  try {
    p = new lma_plan();
    std::string err;
    lma_status s = lma::build_host_plan(optics, lattice, detectors, &p->h, &err);
    if (s != LMA_OK) {
      delete p;
      return fail(s, err);
    }
    p->host_only = (flags & LMA_HOST_ONLY) != 0;
    p->stream = reinterpret_cast<hipStream_t>(hip_stream);
    const HostPlan& h = p->h;
    lma::build_stencil(h, lma::dev::kStencilMaxKs, lma::dev::kStencilMaxRect, &p->st);
    p->B = std::max(1, std::min<int>(auto_batch(h), (int)std::max<int64_t>(std::max<int64_t>((int64_t)h.rows.size(), h.n_probes()), 1)));
    if (!p->host_only && hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return fail(LMA_ERR_DEVICE, "no HIP device");
    }
    if (!p->host_only && ((flags & LMA_OWN_STREAM) || ((flags & LMA_GRAPH) && !p->stream))) {
      // non-blocking: the plan's work never waits for, or holds up, the legacy default stream
      if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(LMA_ERR_DEVICE, "stream creation failed");
      }
      p->own_stream = true;
    }
    p->use_graph = (flags & LMA_GRAPH) != 0;
    if (const char* e = std::getenv("LMA_TILE_WIDTH")) lma::dev::set_tile_width(std::atoi(e));
    p->tw = lma::dev::tile_width(h.op.nx, h.op.ny);
    // a forced radix schedule (tuning and tests), 0 to 2
    if (const char* e = std::getenv("LMA_RADIX_SCHEDULE")) p->sched = std::min(2, std::max(0, std::atoi(e)));
    if (!p->host_only && (flags & LMA_AUTOTUNE)) {
      lma_tuning t{};
      if (lma_status ts = lma_autotune(h.op.nx, h.op.ny, 0, p->stream, &t); ts != LMA_OK) {
        release(p);
        return ts;
      }
      p->tw = t.tile_width;
      p->sched = t.radix_schedule;
      if (h.lat.batch <= 0)
        p->B = std::max(1, std::min<int>(t.batch, (int)std::max<int64_t>(std::max<int64_t>((int64_t)h.rows.size(), h.n_probes()), 1)));
    }
    // residency (Sec. 4.2.4): the whole window's basis, or a rectangle partition when it needs
    // more than M = budget / (D x 8 B) propagated translates
    {
      const int64_t row_bytes = (int64_t)h.D() * 8;
      int64_t max_rows = -1;
      if (h.lat.hbm_budget_bytes > 0) {
        max_rows = h.lat.hbm_budget_bytes / row_bytes;
      } else if (!p->host_only) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
          const int64_t spare = (int64_t)fr - footprint_of(h, p->B, 1, false) - ((int64_t)256 << 20);
          max_rows = std::max<int64_t>(0, spare / row_bytes);
        }
      }
      if (max_rows >= 0 && (int64_t)h.rows.size() > max_rows) {
        std::string why;
        if (!lma::build_partition(h, max_rows, &p->pp, &why)) {
          delete p;
          return fail(LMA_ERR_OOM, why);
        }
        p->partitioned = true;
      }
    }
    compute_gaps(p);
    if (p->host_only) {
      *out = p;
      return LMA_OK;
    }
    const int64_t XY = (int64_t)h.op.nx * h.op.ny;
    // tables; those read by column passes are transposed to [kx][ky]
    const int nx = h.op.nx, ny = h.op.ny;
    std::vector<float2> v((size_t)XY);
    auto to_f2T = [&](const std::vector<cd>& src, double scale) {
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const cd& z = src[(size_t)y * nx + x];
          v[(size_t)x * ny + y] = make_float2((float)(z.real() * scale), (float)(z.imag() * scale));
        }
    };
    to_f2T(h.spec, 1.0 / (double)XY);
    if ((s = upload(p, &p->d_specT, v.data(), v.size())) != LMA_OK) { release(p); return s; }
    if (h.lat.basis_kind == LMA_BASIS_PROBE) {
      p->d_uspecT = p->d_specT;
    } else {
      to_f2T(h.uspec, 1.0 / (double)XY);
      if ((s = upload(p, &p->d_uspecT, v.data(), v.size())) != LMA_OK) { release(p); return s; }
    }
    to_f2T(h.prop, 1.0);
    if ((s = upload(p, &p->d_propT, v.data(), v.size())) != LMA_OK) { release(p); return s; }
    auto twx = twiddles(nx), twy = twiddles(ny);
    if ((s = upload(p, &p->d_twx, twx.data(), twx.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_twy, twy.data(), twy.size())) != LMA_OK) { release(p); return s; }
    if (h.wnx > 0) {
      const int wx = h.wnx, wy = h.wny;
      std::vector<float2> wv((size_t)wx * wy);
      auto wT = [&](const std::vector<cd>& src, double scale) {
        for (int y = 0; y < wy; ++y)
          for (int x = 0; x < wx; ++x) {
            const cd& z = src[(size_t)y * wx + x];
            wv[(size_t)x * wy + y] = make_float2((float)(z.real() * scale), (float)(z.imag() * scale));
          }
      };
      wT(h.wspec, 1.0 / ((double)wx * wy));
      if ((s = upload(p, &p->d_wspecT, wv.data(), wv.size())) != LMA_OK) { release(p); return s; }
      wT(h.wprop, 1.0);
      if ((s = upload(p, &p->d_wpropT, wv.data(), wv.size())) != LMA_OK) { release(p); return s; }
      auto wtx = twiddles(wx), wty = twiddles(wy);
      if ((s = upload(p, &p->d_wtwx, wtx.data(), wtx.size())) != LMA_OK) { release(p); return s; }
      if ((s = upload(p, &p->d_wtwy, wty.data(), wty.size())) != LMA_OK) { release(p); return s; }
      std::vector<int64_t> zeros((size_t)p->B * 2, 0);
      if ((s = upload(p, &p->d_zero_u, zeros.data(), zeros.size())) != LMA_OK) { release(p); return s; }
      if ((s = dalloc(p, (void**)&p->d_wwork, (size_t)p->B * wx * wy * sizeof(float2))) != LMA_OK) { release(p); return s; }
    }
    std::vector<int32_t> compT((size_t)XY);
    std::vector<uint32_t> maskT((size_t)XY);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        compT[(size_t)x * ny + y] = h.comp_map[(size_t)y * nx + x];
        maskT[(size_t)x * ny + y] = h.detmask[(size_t)y * nx + x];
      }
    if ((s = upload(p, &p->d_compT, compT.data(), compT.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_maskT, maskT.data(), maskT.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_row_of, h.row_of.data(), h.row_of.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_set_dx, h.set_dx.data(), h.set_dx.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_set_dy, h.set_dy.data(), h.set_dy.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_chunk_start, h.chunk_start.data(), h.chunk_start.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_chunk_len, h.chunk_len.data(), h.chunk_len.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_chunk_mask, h.chunk_mask.data(), h.chunk_mask.size())) != LMA_OK) { release(p); return s; }
    std::vector<float2> al(h.alpha.size());
    for (size_t i = 0; i < al.size(); ++i) al[i] = make_float2((float)h.alpha[i].real(), (float)h.alpha[i].imag());
    if ((s = upload(p, &p->d_alpha, al.data(), al.size())) != LMA_OK) { release(p); return s; }
    if (p->st.ok) {
      std::vector<float2> sa(p->st.a.size());
      for (size_t i = 0; i < sa.size(); ++i) sa[i] = make_float2(p->st.a[i].real(), p->st.a[i].imag());
      if ((s = upload(p, &p->d_stencil_a, sa.data(), sa.size())) != LMA_OK) { release(p); return s; }
      if ((s = upload(p, &p->d_ks_off, p->st.ks_off.data(), p->st.ks_off.size())) != LMA_OK) { release(p); return s; }
      if (h.lat.precision == LMA_GEMM_SPLIT_BF16) {
        // A fragments of the bf16 MFMA: group G of 4 K-steps, lane l = m + 16 g holds the
        // coefficients of probe m for the 4 translates of K-step 4 G + g, each split into hi
        // and lo bf16 (Re hi x4, Re lo x4, Im hi x4, Im lo x4)
        const int nks = p->st.nks, ng = (nks + 3) / 4;
        std::vector<uint16_t> abf((size_t)ng * 64 * 16, 0);
        for (int G = 0; G < ng; ++G)
          for (int l = 0; l < 64; ++l) {
            const int m = l % 16, g = l / 16, ks = 4 * G + g;
            uint16_t* o = &abf[((size_t)G * 64 + l) * 16];
            for (int i = 0; i < 4 && ks < nks; ++i) {
              const std::complex<float> z = p->st.a[(size_t)ks * 64 + m + 16 * i];
              const uint16_t rh = bf16_round(z.real()), ih = bf16_round(z.imag());
              o[i] = rh;
              o[4 + i] = bf16_round(z.real() - bf16_value(rh));
              o[8 + i] = ih;
              o[12 + i] = bf16_round(z.imag() - bf16_value(ih));
            }
          }
        if ((s = upload(p, &p->d_stencil_abf, abf.data(), abf.size())) != LMA_OK) { release(p); return s; }
      }
    }
    // wave position lists
    std::vector<int64_t> ru(h.rows.size() * 2);
    std::vector<int32_t> rid(h.rows.size());
    for (size_t r = 0; r < h.rows.size(); ++r) {
      int t = h.rows[r];
      ru[2 * r] = ((t % h.Rfx) * h.stepTx + h.oxu) % h.Qx;
      ru[2 * r + 1] = ((t / h.Rfx) * h.stepTy + h.oyu) % h.Qy;
      rid[r] = (int32_t)r;
    }
    if ((s = upload(p, &p->d_row_u, ru.data(), ru.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_row_id, rid.data(), rid.size())) != LMA_OK) { release(p); return s; }
    std::vector<int64_t> pu((size_t)h.n_probes() * 2);
    std::vector<int32_t> po((size_t)h.n_probes());
    for (int b = 0; b < h.wh; ++b)
      for (int a = 0; a < h.ww; ++a) {
        int64_t i = (int64_t)b * h.ww + a;
        pu[2 * i] = ((int64_t)(h.wa0 + a) * h.stepPx) % h.Qx;
        pu[2 * i + 1] = ((int64_t)(h.wb0 + b) * h.stepPy) % h.Qy;
        po[i] = (int32_t)i;
      }
    if ((s = upload(p, &p->d_probe_u, pu.data(), pu.size())) != LMA_OK) { release(p); return s; }
    if ((s = upload(p, &p->d_probe_out, po.data(), po.size())) != LMA_OK) { release(p); return s; }
    // buffers
    if ((s = dalloc(p, (void**)&p->d_img, (size_t)h.ndet * h.n_probes() * sizeof(double))) != LMA_OK) { release(p); return s; }
    {
      const std::vector<float2> z(32, make_float2(0.f, 0.f));
      if ((s = upload(p, &p->d_zeros, z.data(), z.size())) != LMA_OK) { release(p); return s; }
    }
    if ((s = dalloc(p, (void**)&p->d_work, (size_t)p->B * XY * sizeof(float2))) != LMA_OK) { release(p); return s; }
    if (p->partitioned) {
      const lma::PartPlan& pp = p->pp;
      const size_t NT = (size_t)h.n_translates();
      std::vector<int32_t> row_of(pp.parts.size() * NT), slot, probes;
      std::vector<int64_t> u;
      p->part_fresh_off.assign(1, 0);
      p->part_probe_off.assign(1, 0);
      for (size_t j = 0; j < pp.parts.size(); ++j) {
        const lma::PartPlan::Part& q = pp.parts[j];
        std::copy(q.row_of.begin(), q.row_of.end(), row_of.begin() + j * NT);
        for (size_t i = 0; i < q.fresh.size(); ++i) {
          const int t = q.fresh[i];
          u.push_back(((t % h.Rfx) * h.stepTx + h.oxu) % h.Qx);
          u.push_back(((t / h.Rfx) * h.stepTy + h.oyu) % h.Qy);
          slot.push_back(q.fresh_slot[i]);
        }
        p->part_fresh_off.push_back((int64_t)slot.size());
        if (!p->st.ok)
          for (int b = q.b0; b < q.b0 + q.h; ++b)
            for (int a = q.a0; a < q.a0 + q.w; ++a) probes.push_back(b * h.ww + a);
        p->part_probe_off.push_back((int64_t)probes.size());
      }
      if ((s = upload(p, &p->d_part_row_of, row_of.data(), row_of.size())) != LMA_OK) { release(p); return s; }
      if ((s = upload(p, &p->d_part_u, u.data(), u.size())) != LMA_OK) { release(p); return s; }
      if ((s = upload(p, &p->d_part_slot, slot.data(), slot.size())) != LMA_OK) { release(p); return s; }
      if ((s = upload(p, &p->d_part_probes, probes.data(), probes.size())) != LMA_OK) { release(p); return s; }
      if ((s = dalloc(p, &p->d_basis, (size_t)pp.slots * h.D() * 8 + 128)) != LMA_OK) { release(p); return s; }
    } else {
      if ((s = dalloc(p, &p->d_basis, (size_t)h.rows.size() * h.D() * 8 + 128)) != LMA_OK) { release(p); return s; }
    }
    *out = p;
    return LMA_OK;
  } catch (const std::bad_alloc&) {
    if (p) release(p);
    return fail(LMA_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    if (p) release(p);
    return fail(LMA_ERR_ARG, e.what());
  }
}

static lma_status check_device_call(lma_plan* p, const void* ptr, int32_t nslices) {
  if (!p) return fail(LMA_ERR_ARG, "plan is null");
  if (p->host_only) return fail(LMA_ERR_STATE, "host-only plan has no device state");
  if (!ptr) return fail(LMA_ERR_ARG, "null data pointer");
  if (nslices < 1) return fail(LMA_ERR_ARG, "nslices must be >= 1");
  return LMA_OK;
}

lma_status lma_propagate(lma_plan* plan, const float* potential, int32_t nslices, int32_t flags) {
  lma_status s = check_device_call(plan, potential, nslices);
  if (s != LMA_OK) return s;
  if (plan->partitioned)
    return fail(LMA_ERR_STATE, "the window's basis exceeds the residency budget: the plan is partitioned "
                               "into rectangles, use lma_image");
  plan->basis_valid = false;
  try {
    if ((s = prepare_transmission(plan, potential, nslices, flags)) != LMA_OK) return s;
    if ((s = waves(plan, plan->d_row_u, plan->d_row_id, nullptr, (int)plan->h.rows.size(), nslices)) != LMA_OK) return s;
    if (!(flags & LMA_PTR_DEVICE)) HIP_TRY(hipStreamSynchronize(plan->stream));
    plan->basis_valid = true;
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_probe_image(lma_plan* plan, double* image, int32_t flags, double weight) {
  lma_status s = check_device_call(plan, image, 1);
  if (s != LMA_OK) return s;
  if (!plan->basis_valid) return fail(LMA_ERR_STATE, "no valid propagated basis (call lma_propagate)");
  if (!std::isfinite(weight)) return fail(LMA_ERR_ARG, "weight must be finite");
  try {
    HIP_TRY(hipMemsetAsync(plan->d_img, 0, (size_t)plan->h.ndet * plan->h.n_probes() * sizeof(double), plan->stream));
    if (plan->st.ok && !(flags & LMA_CONTRACT_PER_PIXEL))
      LAUNCH(plan, "contract_mfma", lma::dev::contract_stencil(stencil(plan), plan->stream));
    else
      LAUNCH(plan, "contract", lma::dev::contract(contraction(plan), plan->stream));
    return write_image(plan, image, flags, weight);
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_image(lma_plan* plan, const float* potential, int32_t nslices, double* image, int32_t flags,
                     double weight) {
  lma_status s = check_device_call(plan, potential, nslices);
  if (s != LMA_OK) return s;
  if (!image) return fail(LMA_ERR_ARG, "image is null");
  if (!std::isfinite(weight)) return fail(LMA_ERR_ARG, "weight must be finite");
  if (!plan->partitioned) {
    if ((s = lma_propagate(plan, potential, nslices, flags)) != LMA_OK) return s;
    return lma_probe_image(plan, image, flags, weight);
  }
  const HostPlan& h = plan->h;
  plan->basis_valid = false;
  try {
    if ((s = prepare_transmission(plan, potential, nslices, flags)) != LMA_OK) return s;
    HIP_TRY(hipMemsetAsync(plan->d_img, 0, (size_t)h.ndet * h.n_probes() * sizeof(double), plan->stream));
    const size_t NT = (size_t)h.n_translates();
    for (size_t j = 0; j < plan->pp.parts.size(); ++j) {
      const lma::PartPlan::Part& q = plan->pp.parts[j];
      const int64_t f0 = plan->part_fresh_off[j], nf = plan->part_fresh_off[j + 1] - f0;
      // step 1 for the translates this rectangle adds to the resident set
      if (nf > 0 && (s = waves(plan, plan->d_part_u + 2 * f0, plan->d_part_slot + f0, nullptr, (int)nf, nslices)) != LMA_OK)
        return s;
      // step 2 and the detector for the rectangle's probes
      if (plan->st.ok) {
        lma::dev::Stencil c = stencil(plan);
        c.row_of = plan->d_part_row_of + j * NT;
        // the super-tiles (8 x 8 probes, aligned) that meet the rectangle; only the
        // rectangle's probes are added to the image
        c.tile_x0 = q.a0 / 8;
        c.tile_y0 = q.b0 / 8;
        c.tiles_x = (q.a0 + q.w - 1) / 8 - c.tile_x0 + 1;
        c.tiles_y = (q.b0 + q.h - 1) / 8 - c.tile_y0 + 1;
        c.pa0 = q.a0;
        c.pa1 = q.a0 + q.w;
        c.pb0 = q.b0;
        c.pb1 = q.b0 + q.h;
        LAUNCH(plan, "contract_mfma", lma::dev::contract_stencil(c, plan->stream));
      } else {
        lma::dev::Contraction c = contraction(plan);
        c.row_of = plan->d_part_row_of + j * NT;
        c.probe_list = plan->d_part_probes + plan->part_probe_off[j];
        c.n_list = (int)(plan->part_probe_off[j + 1] - plan->part_probe_off[j]);
        LAUNCH(plan, "contract", lma::dev::contract(c, plan->stream));
      }
    }
    return write_image(plan, image, flags, weight);
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_plain_image(lma_plan* plan, const float* potential, int32_t nslices, double* image, int32_t flags,
                           double weight) {
  lma_status s = check_device_call(plan, potential, nslices);
  if (s != LMA_OK) return s;
  if (!image) return fail(LMA_ERR_ARG, "image is null");
  if (!std::isfinite(weight)) return fail(LMA_ERR_ARG, "weight must be finite");
  try {
    if ((s = prepare_transmission(plan, potential, nslices, flags)) != LMA_OK) return s;
    HIP_TRY(hipMemsetAsync(plan->d_img, 0, (size_t)plan->h.ndet * plan->h.n_probes() * sizeof(double), plan->stream));
    if ((s = waves(plan, plan->d_probe_u, nullptr, plan->d_probe_out, (int)plan->h.n_probes(), nslices)) != LMA_OK) return s;
    return write_image(plan, image, flags, weight);
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

}  // extern "C"

// ---- the plain image without allocation ----------------------------------------------------
// Its transmission tables, wave batch and image accumulator live in one file-scope device
// array, so the call makes no allocation. In host code the array's name is a host-side
// stand-in: kernels get its device address, looked up once per device.
namespace {
static __device__ __align__(256) unsigned char scratch[LMA_NOALLOC_SCRATCH_BYTES];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kScratchDevices] = {};

// the scratch array's address on device `dev`, which must be the current device
lma_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kScratchDevices) return fail(LMA_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(LMA_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return LMA_OK;
}

int64_t round256(int64_t b) { return (b + 255) & ~(int64_t)255; }
}  // namespace

extern "C" {

lma_status lma_plain_image_noalloc(lma_plan* plan, const float* potential, int32_t nslices, double* image,
                                   int32_t flags, double weight) {
  lma_status s = check_device_call(plan, potential, nslices);
  if (s != LMA_OK) return s;
  if (!image) return fail(LMA_ERR_ARG, "image is null");
  if (!std::isfinite(weight)) return fail(LMA_ERR_ARG, "weight must be finite");
  if (!(flags & LMA_PTR_DEVICE)) return fail(LMA_ERR_ARG, "lma_plain_image_noalloc takes device pointers only (LMA_PTR_DEVICE)");
  if (flags & ~(int32_t)(LMA_PTR_DEVICE | LMA_ACCUMULATE)) return fail(LMA_ERR_ARG, "unsupported flags");
  const HostPlan& h = plan->h;
  const int64_t XY = (int64_t)h.op.nx * h.op.ny, np = h.n_probes(), n = (int64_t)h.ndet * np;
  const int64_t img_bytes = round256(n * 8), trans_bytes = round256((int64_t)nslices * XY * 8), wave = XY * 8;
  const int64_t cap = (int64_t)LMA_NOALLOC_SCRATCH_BYTES;
  if (img_bytes + trans_bytes + wave > cap)
    return fail(LMA_ERR_ARG, "lma_plain_image_noalloc needs " + std::to_string(img_bytes + trans_bytes + wave) +
                                 " bytes of scratch (image, transmission tables, one wave); the library holds " +
                                 std::to_string(cap));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
    return fail(LMA_ERR_ARG, "call lma_plain_image_noalloc with the plan's device current");
  unsigned char* base = nullptr;
  if ((s = scratch_address(dev, &base)) != LMA_OK) return s;
  WaveBufs wb;
  wb.img = reinterpret_cast<double*>(base);
  wb.trans = reinterpret_cast<const float2*>(base + img_bytes);
  wb.work = reinterpret_cast<float2*>(base + img_bytes + trans_bytes);
  wb.B = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)plan->B, np, (cap - img_bytes - trans_bytes) / wave}));
  try {
    LAUNCH(plan, "fill_zero", lma::dev::fill_zero(wb.img, n, plan->stream));
    LAUNCH(plan, "transmission", lma::dev::transmission(potential, reinterpret_cast<float2*>(base + img_bytes),
                                                        (int64_t)nslices * XY, h.op.sigma, plan->stream));
    if ((s = run_waves(plan, plan->d_probe_u, nullptr, plan->d_probe_out, (int)np, nslices, nullptr, false, &wb)) != LMA_OK)
      return s;
    LAUNCH(plan, "scale_out", lma::dev::scale_out(image, wb.img, n, weight, (flags & LMA_ACCUMULATE) ? 1 : 0, plan->stream));
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_probe_patterns(lma_plan* plan, float* out, int32_t flags) {
  lma_status s = check_device_call(plan, out, 1);
  if (s != LMA_OK) return s;
  if (plan->partitioned) return fail(LMA_ERR_STATE, "the plan is partitioned: its basis is never resident whole");
  if (!plan->basis_valid) return fail(LMA_ERR_STATE, "no valid propagated basis (call lma_propagate)");
  const int64_t n = plan->h.n_probes() * (int64_t)plan->h.D();
  try {
    float* dst = out;
    if (!(flags & LMA_PTR_DEVICE) && (s = dalloc(plan, (void**)&dst, (size_t)n * sizeof(float))) != LMA_OK) return s;
    lma::dev::Contraction c = contraction(plan);
    c.patterns = dst;
    Launch l(plan, "contract_pattern");
    hipError_t e = lma::dev::contract(c, plan->stream);
    l.done();
    if (e == hipSuccess && !(flags & LMA_PTR_DEVICE)) {
      e = hipMemcpyAsync(out, dst, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, plan->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    }
    if (dst != out) free_one(plan, dst, (size_t)n * sizeof(float));
    if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("patterns: ") + hipGetErrorString(e));
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_probe_radial(lma_plan* plan, double width, int32_t nbins, double* image, int32_t flags, double weight) {
  lma_status s = check_device_call(plan, image, 1);
  if (s != LMA_OK) return s;
  if (!(width > 0) || !std::isfinite(width)) return fail(LMA_ERR_ARG, "annulus width must be positive");
  if (nbins < 1 || nbins > lma::dev::kMaxRadialBins) return fail(LMA_ERR_ARG, "nbins must be in [1, 512]");
  if (!std::isfinite(weight)) return fail(LMA_ERR_ARG, "weight must be finite");
  if (plan->partitioned) return fail(LMA_ERR_STATE, "the plan is partitioned: its basis is never resident whole");
  if (!plan->basis_valid) return fail(LMA_ERR_STATE, "no valid propagated basis (call lma_propagate)");
  const HostPlan& h = plan->h;
  const int D = h.D();
  const int64_t n = (int64_t)nbins * h.n_probes();
  try {
    if (!plan->d_bin_of || plan->bin_width != width || plan->bin_count != nbins) {
      // annulus of every detector pixel: a = floor(lambda |k| / width) while below nbins
      std::vector<int32_t> bin(D);
      for (int d = 0; d < D; ++d) {
        const int f = h.comp_flat[d];
        const int mx = f % h.op.nx, my = f / h.op.nx;
        const double kx = (double)(mx < (h.op.nx + 1) / 2 ? mx : mx - h.op.nx) / h.op.lx;
        const double ky = (double)(my < (h.op.ny + 1) / 2 ? my : my - h.op.ny) / h.op.ly;
        const double a = std::floor(h.op.wavelength * std::sqrt(kx * kx + ky * ky) / width);
        bin[d] = a < (double)nbins ? (int32_t)a : -1;
      }
      if (!plan->d_bin_of && (s = dalloc(plan, (void**)&plan->d_bin_of, (size_t)D * sizeof(int32_t))) != LMA_OK) return s;
      HIP_TRY(hipMemcpy(plan->d_bin_of, bin.data(), (size_t)D * sizeof(int32_t), hipMemcpyHostToDevice));
      plan->bin_width = width;
      plan->bin_count = nbins;
    }
    double* acc = nullptr;
    if ((s = dalloc(plan, (void**)&acc, (size_t)n * sizeof(double))) != LMA_OK) return s;
    lma::dev::Contraction c = contraction(plan);
    c.bin_of = plan->d_bin_of;
    c.nbins = nbins;
    c.radial = acc;
    hipError_t e = hipMemsetAsync(acc, 0, (size_t)n * sizeof(double), plan->stream);
    if (e == hipSuccess) {
      Launch l(plan, "contract_radial");
      e = lma::dev::contract(c, plan->stream);
      l.done();
    }
    if (e == hipSuccess && (flags & LMA_PTR_DEVICE)) {
      e = lma::dev::scale_out(image, acc, n, weight, (flags & LMA_ACCUMULATE) ? 1 : 0, plan->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    } else if (e == hipSuccess) {
      std::vector<double> tmp((size_t)n);
      e = hipMemcpyAsync(tmp.data(), acc, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, plan->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
      if (e == hipSuccess)
        for (int64_t i = 0; i < n; ++i) image[i] = (flags & LMA_ACCUMULATE) ? image[i] + weight * tmp[i] : weight * tmp[i];
    }
    free_one(plan, acc, (size_t)n * sizeof(double));
    if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("radial: ") + hipGetErrorString(e));
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_plain_patterns(lma_plan* plan, const float* potential, int32_t nslices, float* out, int32_t flags) {
  lma_status s = check_device_call(plan, potential, nslices);
  if (s != LMA_OK) return s;
  if (!out) return fail(LMA_ERR_ARG, "out is null");
  const int64_t np = plan->h.n_probes(), D = plan->h.D(), n = np * D;
  try {
    if ((s = prepare_transmission(plan, potential, nslices, flags)) != LMA_OK) return s;
    float2* spec = nullptr;
    float* dst = out;
    if ((s = dalloc(plan, (void**)&spec, (size_t)n * sizeof(float2))) != LMA_OK) return s;
    if (!(flags & LMA_PTR_DEVICE) && (s = dalloc(plan, (void**)&dst, (size_t)n * sizeof(float))) != LMA_OK) {
      free_one(plan, spec, (size_t)n * sizeof(float2));
      return s;
    }
    s = run_waves(plan, plan->d_probe_u, plan->d_probe_out, nullptr, (int)np, nslices, spec, true);
    hipError_t e = hipSuccess;
    if (s == LMA_OK) {
      e = lma::dev::intensity(spec, dst, n, (double)plan->h.op.nx * plan->h.op.ny, plan->stream);
      if (e == hipSuccess && !(flags & LMA_PTR_DEVICE))
        e = hipMemcpyAsync(out, dst, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, plan->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    }
    free_one(plan, spec, (size_t)n * sizeof(float2));
    if (dst != out) free_one(plan, dst, (size_t)n * sizeof(float));
    if (s != LMA_OK) return s;
    if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("plain patterns: ") + hipGetErrorString(e));
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_recompute_local(lma_plan* plan, const float* potential_new, int32_t nslices, const int32_t bbox_px[4],
                               double radius_A, double* image, int32_t* n_translates_redone,
                               int32_t* n_probes_redone) {
  lma_status s = check_device_call(plan, potential_new, nslices);
  if (s != LMA_OK) return s;
  if (!image || !bbox_px) return fail(LMA_ERR_ARG, "null argument");
  if (!plan->basis_valid) return fail(LMA_ERR_STATE, "no valid propagated basis (call lma_propagate)");
  if (!std::isfinite(radius_A)) return fail(LMA_ERR_ARG, "radius must be finite");
  const HostPlan& h = plan->h;
  const int nx = h.op.nx, ny = h.op.ny;
  if (bbox_px[2] <= bbox_px[0] || bbox_px[3] <= bbox_px[1]) return fail(LMA_ERR_ARG, "empty edit box");
  try {
    // translates whose centre lies within radius_A of the edited pixels (periodic distance)
    const double dx = h.op.lx / nx, dy = h.op.ly / ny;
    auto axis_dist = [](double c, double lo, double hi, double l) {
      // distance from c to the periodic interval [lo, hi] (hi - lo < l means a proper interval)
      if (hi - lo >= l) return 0.0;
      double t = std::fmod(c - lo, l);
      if (t < 0) t += l;
      double w = hi - lo;
      if (t <= w) return 0.0;
      return std::min(t - w, l - t);
    };
    const double x0 = bbox_px[0] * dx, x1 = (bbox_px[2] - 1) * dx;
    const double y0 = bbox_px[1] * dy, y1 = (bbox_px[3] - 1) * dy;
    std::vector<int32_t> redo_rows;
    std::vector<uint8_t> redo_t((size_t)h.n_translates(), 0);
    for (size_t r = 0; r < h.rows.size(); ++r) {
      int t = h.rows[r];
      double fx, fy;
      h.translate_frac(t, &fx, &fy);
      double ddx = axis_dist(fx * h.op.lx, x0, x1, h.op.lx);
      double ddy = axis_dist(fy * h.op.ly, y0, y1, h.op.ly);
      if (radius_A <= 0 || ddx * ddx + ddy * ddy <= radius_A * radius_A) {
        redo_rows.push_back((int32_t)r);
        redo_t[t] = 1;
      }
    }
    // probes whose L-nearest set meets the re-propagated translates
    std::vector<int32_t> redo_probes;
    for (int b = 0; b < h.wh; ++b)
      for (int a = 0; a < h.ww; ++a) {
        int set, shx, shy;
        h.probe_set(h.wa0 + a, h.wb0 + b, &set, &shx, &shy);
        bool hit = false;
        for (int j = 0; j < h.lat.L && !hit; ++j) {
          int ta = (h.set_dx[(size_t)set * h.lat.L + j] + shx) % h.Rfx;
          int tb = (h.set_dy[(size_t)set * h.lat.L + j] + shy) % h.Rfy;
          hit = redo_t[(size_t)tb * h.Rfx + ta] != 0;
        }
        if (hit) redo_probes.push_back(b * h.ww + a);
      }
    if (n_translates_redone) *n_translates_redone = (int32_t)redo_rows.size();
    if (n_probes_redone) *n_probes_redone = (int32_t)redo_probes.size();
    if (redo_rows.empty()) return LMA_OK;
    plan->basis_valid = false;
    if ((s = prepare_transmission(plan, potential_new, nslices, 0)) != LMA_OK) return s;
    const int n = (int)std::max(redo_rows.size(), redo_probes.size());
    if ((s = ensure_list(plan, n)) != LMA_OK) return s;
    std::vector<int64_t> u(redo_rows.size() * 2);
    for (size_t i = 0; i < redo_rows.size(); ++i) {
      int t = h.rows[redo_rows[i]];
      u[2 * i] = ((t % h.Rfx) * h.stepTx + h.oxu) % h.Qx;
      u[2 * i + 1] = ((t / h.Rfx) * h.stepTy + h.oyu) % h.Qy;
    }
    HIP_TRY(hipMemcpy(plan->d_list_u, u.data(), u.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(plan->d_list, redo_rows.data(), redo_rows.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if ((s = waves(plan, plan->d_list_u, plan->d_list, nullptr, (int)redo_rows.size(), nslices)) != LMA_OK) return s;
    plan->basis_valid = true;
    HIP_TRY(hipStreamSynchronize(plan->stream));
    // re-form the affected probes
    HIP_TRY(hipMemcpy(plan->d_list, redo_probes.data(), redo_probes.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemsetAsync(plan->d_img, 0, (size_t)h.ndet * h.n_probes() * sizeof(double), plan->stream));
    lma::dev::Contraction c = contraction(plan);
    c.probe_list = plan->d_list;
    c.n_list = (int)redo_probes.size();
    LAUNCH(plan, "contract", lma::dev::contract(c, plan->stream));
    std::vector<double> tmp((size_t)h.ndet * h.n_probes());
    HIP_TRY(hipMemcpyAsync(tmp.data(), plan->d_img, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
    const int64_t np = h.n_probes();
    for (int r = 0; r < h.ndet; ++r)
      for (int32_t p : redo_probes) image[r * np + p] = tmp[r * np + p];
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

lma_status lma_synchronize(lma_plan* plan) {
  if (!plan) return fail(LMA_ERR_ARG, "plan is null");
  if (plan->host_only) return LMA_OK;
  hipError_t e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return LMA_OK;
}

lma_status lma_plan_info(const lma_plan* p, lma_info* out) {
  if (!p || !out) return fail(LMA_ERR_ARG, "null argument");
  const HostPlan& h = p->h;
  std::memset(out, 0, sizeof(*out));
  out->nx = h.op.nx;
  out->ny = h.op.ny;
  out->n_translates = (int32_t)h.n_translates();
  out->rfx = h.Rfx;
  out->rfy = h.Rfy;
  out->n_sets = h.nsets;
  out->ncls_x = h.ncls_x;
  out->ncls_y = h.ncls_y;
  out->L = h.lat.L;
  out->n_det = h.ndet;
  out->n_pix = h.D();
  out->n_probes = (int32_t)h.n_probes();
  out->n_rows = (int32_t)h.rows.size();
  out->batch = p->B;
  out->n_aperture = h.n_aperture;
  out->basis_valid = p->basis_valid ? 1 : 0;
  out->host_only = p->host_only ? 1 : 0;
  out->max_residual = h.residual.empty() ? 0.0 : *std::max_element(h.residual.begin(), h.residual.end());
  out->device_bytes = p->dev_bytes;
  out->partitioned = p->partitioned ? 1 : 0;
  out->n_parts = p->partitioned ? (int32_t)p->pp.parts.size() : 1;
  out->part_w = p->partitioned ? p->pp.w : h.ww;
  out->part_h = p->partitioned ? p->pp.h : h.wh;
  out->resident_rows = p->partitioned ? p->pp.slots : (int64_t)h.rows.size();
  out->multislice_calls = p->partitioned ? p->pp.multislice_calls : (int64_t)h.rows.size();
  out->contract_kernel = p->st.ok ? 1 : 0;
  out->contract_k = p->st.ok ? 4 * p->st.nks : (int32_t)h.lat.L;
  out->tile_width = p->tw;
  out->radix_schedule = p->sched;
  out->graphs = p->n_captured;
  out->prop_nx = p->h.wnx;
  out->gap_lo = p->zc0;
  out->gap_hi = p->zc1;
  out->input_gap_lo = p->uc0;
  out->input_gap_hi = p->uc1;
  out->prop_ny = p->h.wny;
  return LMA_OK;
}

lma_status lma_get_translates(const lma_plan* p, double* pos) {
  if (!p || !pos) return fail(LMA_ERR_ARG, "null argument");
  const HostPlan& h = p->h;
  for (int64_t t = 0; t < h.n_translates(); ++t) {
    double fx, fy;
    h.translate_frac((int)t, &fx, &fy);
    pos[2 * t] = fx * h.op.lx;
    pos[2 * t + 1] = fy * h.op.ly;
  }
  return LMA_OK;
}

lma_status lma_get_coefficients(const lma_plan* p, int32_t* translate, double* alpha) {
  if (!p) return fail(LMA_ERR_ARG, "null argument");
  const HostPlan& h = p->h;
  for (size_t i = 0; i < h.set_nbr.size(); ++i) {
    if (translate) translate[i] = h.set_nbr[i];
    if (alpha) {
      alpha[2 * i] = h.alpha[i].real();
      alpha[2 * i + 1] = h.alpha[i].imag();
    }
  }
  return LMA_OK;
}

lma_status lma_get_detector_pixels(const lma_plan* p, int32_t* flat, uint32_t* mask) {
  if (!p) return fail(LMA_ERR_ARG, "null argument");
  const HostPlan& h = p->h;
  for (int d = 0; d < h.D(); ++d) {
    if (flat) flat[d] = h.comp_flat[d];
    if (mask) mask[d] = h.comp_mask[d];
  }
  return LMA_OK;
}

lma_status lma_get_probe_spectrum(const lma_plan* p, double* spec) {
  if (!p || !spec) return fail(LMA_ERR_ARG, "null argument");
  for (size_t i = 0; i < p->h.spec.size(); ++i) {
    spec[2 * i] = p->h.spec[i].real();
    spec[2 * i + 1] = p->h.spec[i].imag();
  }
  return LMA_OK;
}

lma_status lma_get_input_wave_spectrum(const lma_plan* p, double* spec) {
  if (!p || !spec) return fail(LMA_ERR_ARG, "null argument");
  for (size_t i = 0; i < p->h.uspec.size(); ++i) {
    spec[2 * i] = p->h.uspec[i].real();
    spec[2 * i + 1] = p->h.uspec[i].imag();
  }
  return LMA_OK;
}

lma_status lma_get_window_spectrum(const lma_plan* p, double* spec) {
  if (!p || !spec) return fail(LMA_ERR_ARG, "null argument");
  if (p->h.wnx == 0) return fail(LMA_ERR_STATE, "the plan has no translate windows");
  for (size_t i = 0; i < p->h.wspec.size(); ++i) {
    spec[2 * i] = p->h.wspec[i].real();
    spec[2 * i + 1] = p->h.wspec[i].imag();
  }
  return LMA_OK;
}

lma_status lma_get_rows(const lma_plan* p, int32_t* translate) {
  if (!p || !translate) return fail(LMA_ERR_ARG, "null argument");
  std::copy(p->h.rows.begin(), p->h.rows.end(), translate);
  return LMA_OK;
}

// ---- the resident basis as a file --------------------------------------------------------
// Layout: a fixed header, then the rows exactly as the device holds them ([n_rows][D] x 8
// bytes: complex64 scaled by 1/(XY), or four bf16 hi/lo words). The header's fingerprint covers
// everything the rows' values and order depend on besides the potential: the optics, the input
// wave and its translate lattice, the element encoding, the translate windows, the detector
// pixels in compacted order and the resident translates in row order.
namespace {
struct BasisFileHeader {
  char magic[8];
  uint32_t version;
  uint32_t elem_bytes;
  int32_t nx, ny, D, n_rows, precision, reserved;
  uint64_t fingerprint;
  uint64_t payload_bytes;
};
constexpr char kBasisMagic[8] = {'L', 'M', 'A', 'B', 'A', 'S', 'I', 'S'};

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  void put(int32_t v) { bytes(&v, sizeof(v)); }
  void put(double v) { bytes(&v, sizeof(v)); }
};

uint64_t basis_fingerprint(const lma_plan* p) {
  const HostPlan& h = p->h;
  Fnv f;
  f.put(h.op.nx); f.put(h.op.ny); f.put(h.op.lx); f.put(h.op.ly); f.put(h.op.wavelength);
  f.put(h.op.sigma); f.put(h.op.dz); f.put(h.op.bandlimit); f.put(h.op.alpha_max);
  f.put(h.op.defocus); f.put(h.op.cs);
  f.put(h.lat.rx); f.put(h.lat.ry); f.put(h.lat.f); f.put(h.lat.offset_x); f.put(h.lat.offset_y);
  f.put(h.lat.basis_kind); f.put(h.lat.basis_param); f.put(h.lat.precision);
  f.put(h.lat.prop_nx); f.put(h.lat.prop_ny);
  f.bytes(h.comp_flat.data(), h.comp_flat.size() * sizeof(int32_t));
  f.bytes(h.rows.data(), h.rows.size() * sizeof(h.rows[0]));
  return f.h;
}

lma_status basis_file_state(const lma_plan* p) {
  if (p->host_only) return fail(LMA_ERR_STATE, "host-only plan has no device state");
  if (p->partitioned) return fail(LMA_ERR_STATE, "a partitioned plan keeps no whole basis");
  return LMA_OK;
}

constexpr size_t kBasisChunk = (size_t)64 << 20;   // bytes staged through host memory at a time
}  // namespace

lma_status lma_save_basis(lma_plan* p, const char* path) {
  if (!p || !path) return fail(LMA_ERR_ARG, "null argument");
  if (lma_status s = basis_file_state(p); s != LMA_OK) return s;
  if (!p->basis_valid) return fail(LMA_ERR_STATE, "no valid propagated basis");
  BasisFileHeader hd{};
  std::memcpy(hd.magic, kBasisMagic, 8);
  hd.version = 1;
  hd.elem_bytes = 8;
  hd.nx = p->h.op.nx;
  hd.ny = p->h.op.ny;
  hd.D = p->h.D();
  hd.n_rows = (int32_t)p->h.rows.size();
  hd.precision = p->h.lat.precision;
  hd.fingerprint = basis_fingerprint(p);
  hd.payload_bytes = (uint64_t)hd.n_rows * hd.D * hd.elem_bytes;
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(LMA_ERR_ARG, std::string("cannot open for writing: ") + path);
  bool ok = std::fwrite(&hd, sizeof(hd), 1, fp) == 1;
  std::vector<char> buf(std::min<size_t>(kBasisChunk, std::max<uint64_t>(hd.payload_bytes, 1)));
  hipError_t e = hipSuccess;
  for (uint64_t off = 0; ok && off < hd.payload_bytes; off += buf.size()) {
    const size_t n = (size_t)std::min<uint64_t>(buf.size(), hd.payload_bytes - off);
    e = hipMemcpyAsync(buf.data(), (const char*)p->d_basis + off, n, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    ok = e == hipSuccess && std::fwrite(buf.data(), 1, n, fp) == n;
  }
  ok = (std::fclose(fp) == 0) && ok;
  if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("lma_save_basis: ") + hipGetErrorString(e));
  if (!ok) return fail(LMA_ERR_ARG, std::string("write failed: ") + path);
  return LMA_OK;
}

lma_status lma_load_basis(lma_plan* p, const char* path) {
  if (!p || !path) return fail(LMA_ERR_ARG, "null argument");
  if (lma_status s = basis_file_state(p); s != LMA_OK) return s;
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(LMA_ERR_ARG, std::string("cannot open for reading: ") + path);
  BasisFileHeader hd{};
  std::string why;
  if (std::fread(&hd, sizeof(hd), 1, fp) != 1 || std::memcmp(hd.magic, kBasisMagic, 8) != 0)
    why = "not a basis file";
  else if (hd.version != 1 || hd.elem_bytes != 8)
    why = "unsupported basis file version";
  else if (hd.nx != p->h.op.nx || hd.ny != p->h.op.ny || hd.D != p->h.D() ||
           hd.n_rows != (int32_t)p->h.rows.size() || hd.precision != p->h.lat.precision ||
           hd.fingerprint != basis_fingerprint(p) || hd.payload_bytes != (uint64_t)hd.n_rows * hd.D * 8)
    why = "the basis file was written by a plan with another layout (grid, detector pixels, translates, optics or encoding)";
  if (why.empty()) {
    // the payload must be whole before any of it reaches the device
    const long here = std::ftell(fp);
    if (here < 0 || std::fseek(fp, 0, SEEK_END) != 0 || std::ftell(fp) - here != (long)hd.payload_bytes ||
        std::fseek(fp, here, SEEK_SET) != 0)
      why = "the basis file is truncated or has trailing bytes";
  }
  if (!why.empty()) {
    std::fclose(fp);
    return fail(LMA_ERR_ARG, why + ": " + path);
  }
  p->basis_valid = false;
  std::vector<char> buf(std::min<size_t>(kBasisChunk, std::max<uint64_t>(hd.payload_bytes, 1)));
  hipError_t e = hipSuccess;
  bool ok = true;
  for (uint64_t off = 0; off < hd.payload_bytes; off += buf.size()) {
    const size_t n = (size_t)std::min<uint64_t>(buf.size(), hd.payload_bytes - off);
    if (std::fread(buf.data(), 1, n, fp) != n) { ok = false; break; }
    e = hipMemcpyAsync((char*)p->d_basis + off, buf.data(), n, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) break;
  }
  std::fclose(fp);
  if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("lma_load_basis: ") + hipGetErrorString(e));
  if (!ok) return fail(LMA_ERR_ARG, std::string("read failed: ") + path);
  p->basis_valid = true;
  return LMA_OK;
}

lma_status lma_get_basis_rows(lma_plan* p, int32_t first, int32_t count, float* out) {
  if (!p || !out) return fail(LMA_ERR_ARG, "null argument");
  if (p->host_only) return fail(LMA_ERR_STATE, "host-only plan has no device state");
  if (!p->basis_valid) return fail(LMA_ERR_STATE, "no valid propagated basis");
  if (first < 0 || count < 0 || (int64_t)first + count > (int64_t)p->h.rows.size())
    return fail(LMA_ERR_ARG, "row range outside the resident basis");
  const int D = p->h.D();
  const double XY = (double)p->h.op.nx * p->h.op.ny;
  std::vector<uint16_t> raw((size_t)count * D * 4);
  HIP_TRY(hipMemcpyAsync(raw.data(), (const char*)p->d_basis + (size_t)first * D * 8, raw.size() * 2,
                         hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  const bool split = p->h.lat.precision == LMA_GEMM_SPLIT_BF16;
  for (size_t i = 0; i < (size_t)count * D; ++i) {
    float re, im;
    if (split) {
      auto bf = [](uint16_t b) { uint32_t u = (uint32_t)b << 16; float f; std::memcpy(&f, &u, 4); return f; };
      re = bf(raw[4 * i]) + bf(raw[4 * i + 1]);
      im = bf(raw[4 * i + 2]) + bf(raw[4 * i + 3]);
    } else {
      std::memcpy(&re, &raw[4 * i], 4);
      std::memcpy(&im, &raw[4 * i + 2], 4);
    }
    out[2 * i] = (float)(re * XY);
    out[2 * i + 1] = (float)(im * XY);
  }
  return LMA_OK;
}

lma_status lma_set_timing(lma_plan* p, int32_t enable) {
  if (!p) return fail(LMA_ERR_ARG, "plan is null");
  if (p->host_only) return fail(LMA_ERR_STATE, "host-only plan has no device state");
  collect_timing(p);
  if (enable && p->event_pool.size() < kTimingEvents) {
    while (p->event_pool.size() < kTimingEvents) {
      hipEvent_t e = nullptr;
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        (void)hipGetLastError();
        for (hipEvent_t x : p->event_pool) (void)hipEventDestroy(x);
        p->event_pool.clear();
        p->timing = false;
        return fail(LMA_ERR_DEVICE, std::string("timing events: hipEventCreate: ") + hipGetErrorString(err));
      }
      p->event_pool.push_back(e);
    }
  }
  p->timing = enable != 0;
  return LMA_OK;
}

lma_status lma_get_timing(lma_plan* p, lma_kernel_time* out, int32_t max, int32_t* n, int32_t reset) {
  if (!p || !n || (max > 0 && !out)) return fail(LMA_ERR_ARG, "null argument");
  collect_timing(p);
  int k = 0;
  for (auto& t : p->totals) {
    if (k >= max) break;
    std::memset(&out[k], 0, sizeof(lma_kernel_time));
    std::snprintf(out[k].name, sizeof(out[k].name), "%s", t.name.c_str());
    out[k].launches = t.launches;
    out[k].total_ms = t.ms;
    ++k;
  }
  *n = k;
  if (reset) p->totals.clear();
  return LMA_OK;
}

// ---- autotuner ------------------------------------------------------------------------------
namespace {
struct TuneEntry {
  int device, nx, ny;
  int64_t max_bytes;
  lma_tuning t;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

// times one slice (row pass + column pass) per candidate on synthetic waves
lma_status measure_tuning(int nx, int ny, int64_t max_bytes, hipStream_t st, lma_tuning* out) {
  const int64_t XY = (int64_t)nx * ny, wave = XY * (int64_t)sizeof(float2);
  std::vector<int> batches;
  for (int b = 64; b <= 4096; b *= 2)
    if ((int64_t)b * wave <= max_bytes) batches.push_back(b);
  if (batches.empty()) batches.push_back((int)std::max<int64_t>(1, max_bytes / wave));
  std::vector<int> widths;
  for (int tw : {4, 8, 16})
    if (lma::dev::tile_width_ok(nx, ny, tw)) widths.push_back(tw);
  if (widths.empty()) return fail(LMA_ERR_UNSUPPORTED, "no tile width fits this grid");
  std::vector<void*> bufs;
  auto cleanup = [&]() {
    for (void* b : bufs) (void)hipFree(b);
  };
  auto alloc = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    bufs.push_back(q);
    return q;
  };
  float2* work = (float2*)alloc((size_t)batches.back() * wave);
  float2* trans = (float2*)alloc((size_t)wave);
  float2* prop = (float2*)alloc((size_t)wave);
  float2* twx = (float2*)alloc((size_t)nx * sizeof(float2));
  float2* twy = (float2*)alloc((size_t)ny * sizeof(float2));
  hipEvent_t ea = nullptr, eb = nullptr;
  if (!work || !trans || !prop || !twx || !twy) {
    cleanup();
    return fail(LMA_ERR_OOM, "autotune scratch allocation failed");
  }
  std::vector<float2> ones((size_t)XY, make_float2(1.f, 0.f)), scaled((size_t)XY, make_float2(1.f / (float)XY, 0.f));
  auto tx = twiddles(nx), ty = twiddles(ny);
  hipError_t e = hipMemcpy(trans, ones.data(), (size_t)wave, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(prop, scaled.data(), (size_t)wave, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(twx, tx.data(), tx.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(twy, ty.data(), ty.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(work, 0, (size_t)batches.back() * wave, st);
  if (e == hipSuccess) e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  lma_tuning best{};
  best.us_per_wave_slice = 1e300;
  int tried = 0;
  for (int tw : widths) {
    for (int sched = 0; sched < lma::dev::radix_schedules(nx, ny, tw); ++sched)
    for (int B : batches) {
      if (e != hipSuccess) break;
      lma::dev::Tables T;
      T.nx = nx;
      T.ny = ny;
      T.tw = tw;
      T.sched = sched;
      T.propT = prop;
      T.twx = twx;
      T.twy = twy;
      const int reps = 3;
      e = lma::dev::row_pass(T, work, trans, B, true, st);           // warm-up
      if (e == hipSuccess) e = lma::dev::col_pass(T, work, B, st);
      if (e == hipSuccess) e = hipEventRecord(ea, st);
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = lma::dev::row_pass(T, work, trans, B, true, st);
        if (e == hipSuccess) e = lma::dev::col_pass(T, work, B, st);
      }
      if (e == hipSuccess) e = hipEventRecord(eb, st);
      if (e == hipSuccess) e = hipEventSynchronize(eb);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
      if (e != hipSuccess) break;
      ++tried;
      const double us = 1e3 * (double)ms / ((double)reps * B);
      if (us < best.us_per_wave_slice) {
        best.us_per_wave_slice = us;
        best.tile_width = tw;
        best.batch = B;
        best.radix_schedule = sched;
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  cleanup();
  if (e != hipSuccess) return fail(LMA_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  best.candidates = tried;
  *out = best;
  return LMA_OK;
}
}  // namespace

lma_status lma_autotune(int32_t nx, int32_t ny, int64_t max_bytes, void* hip_stream, lma_tuning* out) {
  if (!out) return fail(LMA_ERR_ARG, "out is null");
  if (!lma::dev::supported(nx, ny)) return fail(LMA_ERR_UNSUPPORTED, "the passes are not built for this grid");
  if (max_bytes < 0) return fail(LMA_ERR_ARG, "max_bytes must be >= 0");
  if (max_bytes == 0) max_bytes = (int64_t)4 << 30;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LMA_ERR_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneEntry& t : g_tune)
    if (t.device == dev && t.nx == nx && t.ny == ny && t.max_bytes == max_bytes) {
      *out = t.t;
      return LMA_OK;
    }
  lma_tuning t{};
  lma_status s = measure_tuning(nx, ny, max_bytes, reinterpret_cast<hipStream_t>(hip_stream), &t);
  if (s != LMA_OK) return s;
  g_tune.push_back({dev, nx, ny, max_bytes, t});
  *out = t;
  return LMA_OK;
}

}  // extern "C"

// ---- uneven batch ---------------------------------------------------------------------------
struct lma_batch {
  std::vector<lma_plan*> plans;
  std::vector<int32_t> nslices;
  // grouped batches (lma_batch_create_grouped): plans of one transform-length class hold their
  // translate waves in one buffer, and each row or column pass of a slice is one launch over
  // every wave of the class still propagating
  struct Group {
    std::vector<int> plans;              // indices into `plans`, by decreasing slice count
    std::vector<int64_t> first;          // first wave of each in the group's buffer
    int64_t waves = 0;
    double work = 0.0;                   // pixel-slices of its waves (for balancing branches)
    float2* d_work = nullptr;            // [waves][tiles]
    int32_t* d_wave_spec = nullptr;      // [waves] position in `plans` of the wave's plan
    const float2** d_spec_trans = nullptr;  // [plans] transmission tables of each plan
  };
  std::vector<Group> groups;
  std::vector<int> solo;                 // plans that run their own slice loop
  std::vector<int> branch_of_group, branch_of_solo;
  bool grouped = false;
  hipStream_t origin = nullptr;
  bool own_origin = false;
  std::vector<hipStream_t> branch;   // capture branches
  std::vector<hipEvent_t> plan_ev;   // per plan: its transmission tables are ready
  hipEvent_t fork = nullptr, done = nullptr;
  std::vector<hipEvent_t> join;
  hipGraphExec_t exec = nullptr;
};

namespace {
constexpr int kBatchBranches = 4;

void batch_release(lma_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  for (auto& g : b->groups) {
    if (g.d_work) (void)hipFree(g.d_work);
    if (g.d_wave_spec) (void)hipFree(g.d_wave_spec);
    if (g.d_spec_trans) (void)hipFree(g.d_spec_trans);
  }
  for (hipEvent_t e : b->plan_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->done) (void)hipEventDestroy(b->done);
  for (hipStream_t s : b->branch) (void)hipStreamDestroy(s);
  if (b->own_origin && b->origin) (void)hipStreamDestroy(b->origin);
  delete b;
}

// The slice loop of a group (the translates of every plan in it): each plan's initial waves
// into its part of the buffer, then per slice one row pass over the waves of every plan that
// has the slice (plans sorted by decreasing slice count, so those waves are a prefix), one
// column pass over the waves that go on, and the gather of each plan whose last slice it was.
lma_status run_group(lma_batch* b, const lma_batch::Group& g, hipStream_t st) {
  lma_plan* p0 = b->plans[g.plans[0]];
  const lma::dev::Tables T = tables(p0);
  const int64_t XY = (int64_t)T.nx * T.ny;
  const size_t np = g.plans.size();
  auto check = [](hipError_t e, const char* what) -> lma_status {
    return e == hipSuccess ? LMA_OK : fail(LMA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  lma_status s = LMA_OK;
  // the first row pass skips only the columns every plan's initial waves left zero
  lma::dev::Tables Tr = T;
  Tr.ic0 = 0;
  Tr.ic1 = T.nx;
  for (size_t k = 0; k < np && s == LMA_OK; ++k) {
    lma_plan* p = b->plans[g.plans[k]];
    lma::dev::Tables Ti = tables(p);
    Ti.specT = p->d_uspecT;
    Ti.ic0 = p->uc0;
    Ti.ic1 = p->uc1;
    Tr.ic0 = std::max(Tr.ic0, p->uc0);
    Tr.ic1 = std::min(Tr.ic1, p->uc1);
    s = check(lma::dev::init_waves(Ti, g.d_work + g.first[k] * XY, p->d_row_u, (int)p->h.rows.size(), st), "init");
  }
  if (Tr.ic1 <= Tr.ic0) Tr.ic0 = Tr.ic1 = 0;
  const int maxns = b->nslices[g.plans[0]];
  // waves of the plans with more than j slices
  auto waves_beyond = [&](int j) -> int64_t {
    for (size_t k = 0; k < np; ++k)
      if (b->nslices[g.plans[k]] <= j) return g.first[k];
    return g.waves;
  };
  for (int j = 0; j < maxns && s == LMA_OK; ++j) {
    const int64_t W = waves_beyond(j), Wn = waves_beyond(j + 1);
    s = check(lma::dev::row_pass_specimens(j == 0 ? Tr : T, g.d_work, g.d_spec_trans, g.d_wave_spec, (int64_t)j * XY,
                                           (int)W, j > 0, st),
              "row_pass");
    if (s == LMA_OK && Wn > 0) s = check(lma::dev::col_pass(T, g.d_work, (int)Wn, st), "col_pass");
    for (size_t k = 0; k < np && s == LMA_OK; ++k) {
      if (b->nslices[g.plans[k]] != j + 1) continue;
      lma_plan* p = b->plans[g.plans[k]];
      const int split = p->h.lat.precision == LMA_GEMM_SPLIT_BF16;
      s = check(lma::dev::col_gather(tables(p), g.d_work + g.first[k] * XY, (int)p->h.rows.size(), p->d_basis,
                                     p->h.D(), p->d_row_id, split, st),
                "col_gather");
    }
  }
  return s;
}

// captures every plan's slice loop, plan i on branch i % kBatchBranches; in a grouped batch,
// group k on branch k % kBatchBranches and the plans outside groups after them
lma_status batch_capture(lma_batch* b) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->origin, hipStreamCaptureModeRelaxed));
  lma_status s = LMA_OK;
  hipError_t e = hipEventRecord(b->fork, b->origin);
  for (hipStream_t br : b->branch)
    if (e == hipSuccess) e = hipStreamWaitEvent(br, b->fork, 0);
  for (size_t k = 0; k < b->groups.size() && e == hipSuccess && s == LMA_OK; ++k)
    s = run_group(b, b->groups[k], b->branch[b->branch_of_group[k] % b->branch.size()]);
  std::vector<int> order;
  if (b->grouped) {
    order = b->solo;
  } else {
    for (size_t i = 0; i < b->plans.size(); ++i) order.push_back((int)i);
  }
  for (size_t q = 0; q < order.size() && e == hipSuccess && s == LMA_OK; ++q) {
    lma_plan* p = b->plans[order[q]];
    const hipStream_t keep = p->stream;
    const bool timing = p->timing;
    p->stream = b->branch[(b->grouped ? b->branch_of_solo[q] : (int)q) % b->branch.size()];
    p->timing = false;
    s = run_waves(p, p->d_row_u, p->d_row_id, nullptr, (int)p->h.rows.size(), b->nslices[order[q]]);
    p->stream = keep;
    p->timing = timing;
  }
  for (size_t k = 0; k < b->branch.size() && e == hipSuccess; ++k) {
    e = hipEventRecord(b->join[k], b->branch[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->origin, b->join[k], 0);
  }
  hipError_t ee = hipStreamEndCapture(b->origin, &g);
  if (s != LMA_OK || e != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (s != LMA_OK) return s;
    return fail(LMA_ERR_DEVICE, std::string("batch capture: ") + hipGetErrorString(e != hipSuccess ? e : ee));
  }
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return fail(LMA_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return LMA_OK;
}
}  // namespace

extern "C" {

lma_status lma_batch_create(lma_plan* const* plans, int32_t n, const int32_t* nslices, void* hip_stream,
                            lma_batch** out) {
  if (!out) return fail(LMA_ERR_ARG, "out is null");
  *out = nullptr;
  if (!plans || !nslices || n < 1) return fail(LMA_ERR_ARG, "plans, nslices and n >= 1 required");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LMA_ERR_DEVICE, "no HIP device");
  for (int32_t i = 0; i < n; ++i) {
    lma_plan* p = plans[i];
    if (!p) return fail(LMA_ERR_ARG, "null plan");
    if (p->host_only) return fail(LMA_ERR_STATE, "host-only plan has no device state");
    if (p->partitioned) return fail(LMA_ERR_STATE, "partitioned plans are formed rectangle by rectangle (lma_image)");
    if (p->device != dev) return fail(LMA_ERR_ARG, "every plan must live on the current device");
    if (nslices[i] < 1) return fail(LMA_ERR_ARG, "nslices must be >= 1");
    for (int32_t k = 0; k < i; ++k)
      if (plans[k] == p) return fail(LMA_ERR_ARG, "a plan appears twice");
  }
  lma_batch* b = new lma_batch();
  b->plans.assign(plans, plans + n);
  b->nslices.assign(nslices, nslices + n);
  b->origin = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  if (!b->origin) {
    e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
    b->own_origin = e == hipSuccess;
  }
  for (int k = 0; k < std::min<int>(kBatchBranches, n) && e == hipSuccess; ++k) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) b->branch.push_back(s);
  }
  for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->plan_ev.push_back(ev);
  }
  for (size_t k = 0; k < b->branch.size() && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->join.push_back(ev);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    batch_release(b);
    return fail(LMA_ERR_DEVICE, std::string("batch streams and events: ") + hipGetErrorString(e));
  }
  for (int32_t i = 0; i < n; ++i) {
    lma_status s = ensure_trans(plans[i], nslices[i]);
    if (s != LMA_OK) {
      batch_release(b);
      return s;
    }
  }
  *out = b;
  return LMA_OK;
}

lma_status lma_batch_create_grouped(lma_plan* const* plans, int32_t n, const int32_t* nslices, void* hip_stream,
                                    int64_t max_group_bytes, lma_batch** out) {
  lma_status s = lma_batch_create(plans, n, nslices, hip_stream, out);
  if (s != LMA_OK) return s;
  lma_batch* b = *out;
  b->grouped = true;
  if (max_group_bytes <= 0) max_group_bytes = (int64_t)32 << 30;
  try {
    // a class: same grid, tile width and band gap, bitwise the same propagator table, no
    // translate windows
    std::vector<std::vector<float2>> prop(n);
    auto same_class = [&](int i, int k) {
      const lma_plan *a = plans[i], *c = plans[k];
      if (a->h.op.nx != c->h.op.nx || a->h.op.ny != c->h.op.ny || a->tw != c->tw || a->zc0 != c->zc0 ||
          a->zc1 != c->zc1 || a->pz34 != c->pz34)
        return false;
      return std::memcmp(prop[i].data(), prop[k].data(), prop[i].size() * sizeof(float2)) == 0;
    };
    std::vector<int> cls(n, -1);
    std::vector<std::vector<int>> classes;
    for (int32_t i = 0; i < n; ++i) {
      lma_plan* p = plans[i];
      const int64_t XY = (int64_t)p->h.op.nx * p->h.op.ny;
      const int64_t bytes = (int64_t)p->h.rows.size() * XY * (int64_t)sizeof(float2);
      if (p->h.wnx > 0 || p->h.rows.empty() || bytes > max_group_bytes) {
        b->solo.push_back(i);
        continue;
      }
      prop[i].resize((size_t)XY);
      if (hipMemcpy(prop[i].data(), p->d_propT, (size_t)XY * sizeof(float2), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        throw std::runtime_error("reading a propagator table");
      }
      for (size_t c = 0; c < classes.size() && cls[i] < 0; ++c)
        if (same_class(i, classes[c][0])) cls[i] = (int)c;
      if (cls[i] < 0) {
        cls[i] = (int)classes.size();
        classes.emplace_back();
      }
      classes[cls[i]].push_back(i);
    }
    // groups: a class's plans by decreasing slice count, split where the buffer would exceed
    // max_group_bytes or the group's work would pass an eighth of the batch's (so that the
    // graph's four branches can be balanced)
    auto work_of = [&](int i) {
      return (double)plans[i]->h.rows.size() * plans[i]->h.op.nx * plans[i]->h.op.ny * nslices[i];
    };
    double total = 0.0;
    for (int32_t i = 0; i < n; ++i) total += work_of(i);
    const double target = total / (2.0 * kBatchBranches);
    for (auto& c : classes) {
      std::stable_sort(c.begin(), c.end(), [&](int x, int y) { return nslices[x] > nslices[y]; });
      const int64_t XY = (int64_t)plans[c[0]]->h.op.nx * plans[c[0]]->h.op.ny;
      lma_batch::Group g;
      for (int i : c) {
        const int64_t w = (int64_t)plans[i]->h.rows.size();
        if (!g.plans.empty() &&
            ((g.waves + w) * XY * (int64_t)sizeof(float2) > max_group_bytes || g.work >= target)) {
          b->groups.push_back(std::move(g));
          g = lma_batch::Group();
        }
        g.plans.push_back(i);
        g.first.push_back(g.waves);
        g.waves += w;
        g.work += work_of(i);
      }
      if (!g.plans.empty()) b->groups.push_back(std::move(g));
    }
    // branches: the largest work first, each to the least loaded branch
    {
      std::vector<std::pair<double, int>> items;   // (work, group k >= 0 or solo ~q)
      for (size_t k = 0; k < b->groups.size(); ++k) items.push_back({b->groups[k].work, (int)k});
      for (size_t q = 0; q < b->solo.size(); ++q) items.push_back({work_of(b->solo[q]), ~(int)q});
      std::stable_sort(items.begin(), items.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      std::vector<double> load(kBatchBranches, 0.0);
      b->branch_of_group.assign(b->groups.size(), 0);
      b->branch_of_solo.assign(b->solo.size(), 0);
      for (const auto& it : items) {
        const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[br] += it.first;
        if (it.second >= 0) b->branch_of_group[it.second] = br;
        else b->branch_of_solo[~it.second] = br;
      }
    }
    for (auto& g : b->groups) {
      const lma_plan* p0 = plans[g.plans[0]];
      const int64_t XY = (int64_t)p0->h.op.nx * p0->h.op.ny;
      if (g.waves > (int64_t)INT32_MAX / std::max(1, p0->h.op.ny)) throw std::runtime_error("group too large");
      std::vector<int32_t> spec((size_t)g.waves);
      std::vector<const float2*> trans(g.plans.size());
      for (size_t k = 0; k < g.plans.size(); ++k) {
        const int64_t end = k + 1 < g.plans.size() ? g.first[k + 1] : g.waves;
        std::fill(spec.begin() + g.first[k], spec.begin() + end, (int32_t)k);
        trans[k] = plans[g.plans[k]]->d_trans;
      }
      hipError_t e = hipMalloc((void**)&g.d_work, (size_t)(g.waves * XY) * sizeof(float2));
      if (e == hipSuccess) e = hipMalloc((void**)&g.d_wave_spec, spec.size() * sizeof(int32_t));
      if (e == hipSuccess) e = hipMalloc((void**)&g.d_spec_trans, trans.size() * sizeof(float2*));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        batch_release(b);
        *out = nullptr;
        return fail(LMA_ERR_OOM, std::string("group wave buffer: ") + hipGetErrorString(e));
      }
      e = hipMemcpy(g.d_wave_spec, spec.data(), spec.size() * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy((void*)g.d_spec_trans, trans.data(), trans.size() * sizeof(float2*), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::runtime_error(std::string("group tables: ") + hipGetErrorString(e));
      }
    }
  } catch (const std::exception& ex) {
    batch_release(b);
    *out = nullptr;
    return fail(LMA_ERR_DEVICE, ex.what());
  }
  return LMA_OK;
}

lma_status lma_batch_propagate(lma_batch* b, const float* const* potentials, int32_t flags) {
  if (!b || !potentials) return fail(LMA_ERR_ARG, "null argument");
  for (size_t i = 0; i < b->plans.size(); ++i)
    if (!potentials[i]) return fail(LMA_ERR_ARG, "null potential");
  try {
    lma_status s;
    for (size_t i = 0; i < b->plans.size(); ++i) {
      lma_plan* p = b->plans[i];
      p->basis_valid = false;
      if (b->nslices[i] > p->trans_cap) return fail(LMA_ERR_STATE, "transmission tables were released");
      const float2* keep = p->d_trans;
      if ((s = prepare_transmission(p, potentials[i], b->nslices[i], flags)) != LMA_OK) return s;
      if (p->d_trans != keep) return fail(LMA_ERR_STATE, "transmission tables moved");
      HIP_TRY(hipEventRecord(b->plan_ev[i], p->stream));
      HIP_TRY(hipStreamWaitEvent(b->origin, b->plan_ev[i], 0));
    }
    if (!b->exec && (s = batch_capture(b)) != LMA_OK) return s;
    HIP_TRY(hipGraphLaunch(b->exec, b->origin));
    HIP_TRY(hipEventRecord(b->done, b->origin));
    for (lma_plan* p : b->plans) {
      HIP_TRY(hipStreamWaitEvent(p->stream, b->done, 0));
      p->basis_valid = true;
    }
    if (!(flags & LMA_PTR_DEVICE)) HIP_TRY(hipStreamSynchronize(b->origin));
    return LMA_OK;
  } catch (const std::exception& e) {
    return fail(LMA_ERR_DEVICE, e.what());
  }
}

void lma_batch_destroy(lma_batch* b) {
  if (!b) return;
  if (b->origin) (void)hipStreamSynchronize(b->origin);
  batch_release(b);
}

}  // extern "C"

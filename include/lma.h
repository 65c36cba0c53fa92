/*
 * lma.h -- C ABI of liblma.so, the MI355X (gfx950) hot path of the Lattice Multislice
 * Algorithm (LMA) for STEM image simulation (Doberstein & Binev, "Lattice Multislice
 * Algorithm for Fast Simulation of Scanning Transmission Electron Microscopy Images").
 *
 * Conventions shared by every entry point
 *  - Ownership: callers own every pointer they pass; the library only borrows it for the
 *    duration of the call (device pointers: until the call's stream work completes). A plan
 *    owns every device buffer it allocates (tables, coefficients, the resident propagated
 *    basis) and frees them in lma_destroy.
 *  - Pointers: host pointers unless LMA_PTR_DEVICE is set in `flags`; device pointers must
 *    be on the plan's device.
 *  - Streams: all device work of a plan is ordered on the hipStream_t given to
 *    lma_build_basis (NULL = the legacy default stream). Calls that read or write host
 *    memory synchronise that stream before returning; calls on device memory are
 *    stream-ordered and return before the work completes.
 *  - Errors: no exception or abort crosses the ABI. Every call validates its arguments
 *    before any device work and returns an lma_status; lma_last_error() gives a message
 *    for the calling thread's last non-OK status. A failed lma_propagate marks the
 *    resident basis invalid: lma_probe_image returns LMA_ERR_STATE until a propagate
 *    succeeds.
 *  - Threads: a plan is not thread-safe; separate plans may run concurrently on separate
 *    streams.
 *  - Units: lengths in Angstrom, angles in radians, potentials in V*Angstrom (projected
 *    potential of one slice), the interaction constant in rad/(V*Angstrom).
 *  - Layouts: row-major, x fastest. Complex numbers are interleaved (re, im).
 *  - Transforms: forward DFT F(psi)[k] = sum_x psi[x] exp(-2 pi i k.x); frequencies in
 *    FFT order (k = m/l for m < X/2, (m - X)/l otherwise).
 */
#ifndef LMA_H
#define LMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LMA_OK = 0,
  LMA_ERR_ARG = -1,          /* invalid argument; nothing was done                   */
  LMA_ERR_OOM = -2,          /* device or host allocation failed / over the budget   */
  LMA_ERR_DEVICE = -3,       /* a HIP call failed                                    */
  LMA_ERR_STATE = -4,        /* the plan cannot do this now (no valid basis, host-only plan) */
  LMA_ERR_UNSUPPORTED = -5   /* valid request outside what the library implements    */
} lma_status;

typedef struct lma_plan lma_plan;   /* opaque */

/* lma_lattice.basis_kind: the input wave u whose translates are propagated (Sec. 4.2.3) */
enum {
  LMA_BASIS_PROBE = 0,      /* u = psi_0^init, the probe at the origin                      */
  LMA_BASIS_GAUSSIAN = 1,   /* u = g_sigma(x) = exp(-|x|^2 / (2 sigma^2)), sigma = basis_param */
                            /* (Angstrom; 0 selects lambda / (2 alpha_max))                  */
  LMA_BASIS_TRIGPOLY = 2    /* u(x, y) = phi_nx(2 pi x / lx) phi_ny(2 pi y / ly), the tensor   */
                            /* product of localised trigonometric polynomials (Sec. 2, eq.   */
                            /* rauhut) with the cell as their period; I_f must have 2n + 1   */
                            /* points per axis (odd, at most the grid side), which fixes the */
                            /* degrees. The translates span the frequencies |m| <= n, and the */
                            /* coefficients are the closed form of Sec. 2 (M^-1 per axis), no */
                            /* least squares: exact for probes inside that range when L =    */
                            /* |I_f|; kept at the L nearest translates otherwise             */
};
/* lma_lattice.precision: arithmetic of the probe-coefficient contraction */
enum { LMA_GEMM_FP32 = 0, LMA_GEMM_SPLIT_BF16 = 1 };
/* flags */
enum {
  LMA_PTR_DEVICE = 1,        /* pointer arguments are device pointers                */
  LMA_ACCUMULATE = 2,        /* image += weight * I instead of image = weight * I     */
  LMA_HOST_ONLY = 4,         /* lma_build_basis: plan on the host, no device work     */
  LMA_CONTRACT_PER_PIXEL = 8,/* lma_probe_image: per-pixel VALU contraction even where  */
                             /* the banded MFMA GEMM applies (a cross-check)          */
  LMA_OWN_STREAM = 16,       /* lma_build_basis: the plan creates its own non-blocking */
                             /* stream (default priority) and destroys it with the plan */
  LMA_AUTOTUNE = 32,         /* lma_build_basis: tile width (and the batch, if         */
                             /* lattice.batch is 0) from lma_autotune for this grid    */
  LMA_GRAPH = 64             /* lma_build_basis: a wave sequence (the slice loop of a  */
                             /* batch list) seen a second time with the same buffers is */
                             /* captured into a HIP graph and replayed from then on; a  */
                             /* plan given no stream gets its own (LMA_OWN_STREAM)      */
};

/* Microscope and grid: eqs. probe_wave_function, aberration_function, aperture_function,
 * schroedinger_equation and Sec. 3.2 of the paper. */
typedef struct {
  int32_t nx, ny;            /* X x Y grid: powers of two in [16, 2048], or 96, 192, 384, 640 */
  double lx, ly;             /* periodic cell lx x ly (lx != ly allowed)             */
  double wavelength;         /* lambda                                               */
  double sigma;              /* interaction constant                                 */
  double dz;                 /* slice thickness epsilon                              */
  double bandlimit;          /* |k| < bandlimit * min(X/(2 lx), Y/(2 ly)), in (0, 1]  */
  double alpha_max;          /* aperture: A(k) = 1 iff lambda |k| < alpha_max         */
  double defocus;            /* Z in chi(k) = 1/2 pi Cs lambda^3 |k|^4 - pi Z lambda |k|^2 */
  double cs;                 /* C_s                                                   */
} lma_optics;

/* Probe lattice P, input-wave lattice I and its sublattice I_f, nearest-translate count L
 * (Sec. 4.2.1, options (i) and (iii); Sec. 4.2.2). */
typedef struct {
  int32_t px, py;            /* scan Px x Py, probe a at (a lx/Px, b ly/Py)          */
  int32_t rx, ry;            /* I has Rx x Ry points at spacing r = l/R              */
  int32_t f;                 /* I_f keeps every f-th point of I; R % f == 0           */
  double offset_x, offset_y; /* I_offset as a fraction of r; must be a multiple of
                                1/(2 lcm(P, R)) of the cell                           */
  int32_t L;                 /* nearest translates per probe, 1 <= L <= |I_f|         */
  int32_t basis_kind;        /* LMA_BASIS_PROBE or LMA_BASIS_GAUSSIAN                 */
  int32_t precision;         /* LMA_GEMM_FP32 | LMA_GEMM_SPLIT_BF16                  */
  int32_t window[4];         /* scan window a0, b0, width, height (0,0,0,0 = all)    */
  int32_t batch;             /* waves per propagation batch (0 = automatic)          */
  int64_t hbm_budget_bytes;  /* bytes the resident basis may hold: M = budget/(D x 8) */
                             /* propagated translates (Sec. 4.2.4); 0 = what free     */
                             /* device memory holds after the plan's other buffers    */
  double basis_param;        /* LMA_BASIS_GAUSSIAN: sigma in Angstrom (0: default)     */
  int32_t prop_nx, prop_ny;  /* option (ii) of Sec. 4.2.1: propagate every translate on a */
                             /* prop_nx x prop_ny pixel window centred on it, with the   */
                             /* potential cropped to the window (sides as for nx, ny, at */
                             /* most the grid's; translates must lie on pixels);          */
                             /* 0, 0 = the whole cell                                     */
} lma_lattice;

/* 2-D STEM detectors (Sec. 3.1, step 3): ring r collects lambda|k| in [inner, outer). */
typedef struct {
  int32_t n;                 /* 1..8                                                 */
  const double* inner;       /* [n], radians, >= 0                                   */
  const double* outer;       /* [n], radians, > inner                                */
} lma_detectors;

/* Summary of a built plan. */
typedef struct {
  int32_t nx, ny;
  int32_t n_translates;      /* |I_f|                                                */
  int32_t rfx, rfy;          /* I_f is Rfx x Rfy                                     */
  int32_t n_sets;            /* coefficient sets (Case 1: 1, Case 2: c d)             */
  int32_t ncls_x, ncls_y;    /* sets along x and y                                   */
  int32_t L;
  int32_t n_det;
  int32_t n_pix;             /* D: detector pixels kept per exit wave                */
  int32_t n_probes;          /* probes in the window                                 */
  int32_t n_rows;            /* translates the window needs (resident basis rows)    */
  int32_t batch;             /* waves per propagation batch                          */
  int32_t n_aperture;        /* |K|, frequencies inside the aperture                 */
  int32_t basis_valid;       /* 1 after a successful lma_propagate                   */
  int32_t host_only;
  double max_residual;       /* largest relative LSQ residual over the sets          */
  int64_t device_bytes;      /* device memory held by the plan                       */
  int32_t contract_kernel;   /* window contraction: 1 = banded complex GEMM on MFMA   */
                             /* (4 x 4-probe sub-blocks), 0 = per-pixel VALU sums      */
  int32_t contract_k;        /* translates per probe the contraction multiplies:      */
                             /* 4 x K-steps for MFMA (of which L are non-zero), L else */
  int32_t partitioned;       /* 1: the window is formed in rectangles (lma_image)     */
  int32_t n_parts;           /* rectangles P_1..P_l (1 when not partitioned)          */
  int32_t part_w, part_h;    /* rectangle size in probes (edge ones clipped)           */
  int64_t resident_rows;     /* basis rows held on the device                         */
  int64_t multislice_calls;  /* translates propagated per image: T_{P_1..P_l}         */
  int32_t tile_width;        /* waves are stored in tile_width^2-pixel tiles          */
  int32_t graphs;            /* wave sequences captured as HIP graphs so far          */
  int32_t prop_nx, prop_ny;  /* translate window (0, 0: the whole cell)              */
  int32_t gap_lo, gap_hi;    /* kx columns [gap_lo, gap_hi) where the propagator with  */
                             /* its band limit (Fig. multislice_pseudocode) vanishes  */
                             /* for every ky and no detector pixel lies: waves are    */
                             /* exactly zero there after every propagator multiply,   */
                             /* and the slice passes skip the tile columns inside it  */
  int32_t input_gap_lo, input_gap_hi; /* kx columns where the input wave u's spectrum     */
                             /* vanishes for every ky: the initial-wave pass skips    */
                             /* their tile columns and the first row pass reads none  */
  int32_t radix_schedule;    /* order of the transforms' radices: 0 the base order    */
                             /* (radix 8 first, or the odd radix first), 1 its last   */
                             /* stage first, 2 its first stage last (lma_tuning); -1  */
                             /* each length's default (640: 2, the others 0)           */
} lma_info;

/* Result of lma_autotune for one grid. */
typedef struct {
  int32_t tile_width;        /* fastest tile width of the wave layout (4, 8 or 16)    */
  int32_t batch;             /* fastest waves per propagation batch                  */
  double us_per_wave_slice;  /* its time for one slice (row + column pass) per wave  */
  int32_t candidates;        /* (tile width, batch, radix schedule) triples timed     */
  int32_t radix_schedule;    /* fastest order of the radices (see lma_info); lengths  */
                             /* 256, 384, 640, 1024 and 2048 are built with three     */
} lma_tuning;

/* Per-kernel timing of the last timed calls (enable with lma_set_timing). */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} lma_kernel_time;

/* Relativistic electron wavelength (Angstrom) and interaction constant (rad/(V*A)) for an
 * accelerating voltage in kV (textbook formulas; the paper prints lambda(200 kV) =
 * 0.0250793 A). Either output pointer may be NULL. LMA_ERR_ARG if kv <= 0. */
lma_status lma_electron_constants(double kv, double* wavelength, double* sigma);

/* Plan an LMA simulation (initialisation step of Fig. lma_pseudocode): probe spectrum
 * (eq. probe_wave_function), propagator, detector pixel list, the input-wave lattice I_f,
 * the L nearest translates of every coefficient set and their least-squares coefficients
 * (Sec. 4.2.2, computed on the host in FP64), and the translates the scan window needs.
 * Uploads the tables and allocates the resident basis unless flags has LMA_HOST_ONLY.
 * hip_stream: a hipStream_t (may be NULL; ignored with LMA_OWN_STREAM). On success *out
 * owns the plan. */
lma_status lma_build_basis(const lma_optics* optics, const lma_lattice* lattice,
                           const lma_detectors* detectors, void* hip_stream, int32_t flags,
                           lma_plan** out);

/* Step 1 of Fig. lma_pseudocode: multislice (Fig. multislice_pseudocode) of every needed
 * translate u_i = u(. - i): per slice, transmission by exp(i sigma v_j), forward FFT,
 * Fresnel propagator with band limit, inverse FFT; the exit wave is kept in Fourier
 * space at the D detector pixels as the resident basis.
 * potential: float [nslices][ny][nx] (host, or device with LMA_PTR_DEVICE).
 * Phase arguments sigma*v are formed in FP64. */
lma_status lma_propagate(lma_plan* plan, const float* potential, int32_t nslices, int32_t flags);

/* Step 2 of Fig. lma_pseudocode plus the detector: for every probe p in the window,
 * psi_p^exit = sum_j alpha_{s(p),j} U_{i_j(p)} (eqs. lma_approximation_exit1/2) and
 * I_r(p) = sum over ring r of |F(psi_p^exit)|^2 / (XY).
 * image: double [n_det][h][w] of the window; image = weight*I, or += with LMA_ACCUMULATE
 * (frozen-phonon averaging: weight = 1/n_phonons). Needs a valid basis.
 * The combination runs as a banded complex GEMM on MFMA (FP32 products, FP32 sums over the
 * neighbours, FP64 ring sums) when lma_info.contract_kernel is 1, else (or with
 * LMA_CONTRACT_PER_PIXEL) as per-pixel sums on the vector units; both give the same
 * result up to FP32 rounding order. */
lma_status lma_probe_image(lma_plan* plan, double* image, int32_t flags, double weight);

/* The whole LMA image of the window in one call (steps 1 and 2 of Fig. lma_pseudocode and
 * the detector). A plan whose window needs more propagated translates than the residency
 * budget holds is partitioned at lma_build_basis (lma_info.partitioned = 1) into rectangles
 * of probes P_1..P_l (Sec. 4.2.4, rectangle strategy, row-major): for each rectangle the
 * translates it shares with the previous one stay resident, the others are propagated into
 * the freed rows, then the rectangle's probes are formed; lma_info.multislice_calls gives
 * the number of propagated translates, T_{P_1..P_l}. Such a plan has no complete resident
 * basis: lma_propagate, lma_probe_image and lma_recompute_local return LMA_ERR_STATE. On a
 * plan that is not partitioned this equals lma_propagate followed by lma_probe_image.
 * potential, image, flags and weight as for lma_plain_image. */
lma_status lma_image(lma_plan* plan, const float* potential, int32_t nslices, double* image,
                     int32_t flags, double weight);

/* Plain multislice comparator (Sec. 3.1 steps 1-3): every probe of the window propagated
 * directly, same kernels, same detectors, same image layout and flags as lma_probe_image.
 * Does not touch the resident basis. */
lma_status lma_plain_image(lma_plan* plan, const float* potential, int32_t nslices,
                           double* image, int32_t flags, double weight);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. lma_plain_image with device pointers only
 * (LMA_PTR_DEVICE required; LMA_ACCUMULATE optional), making no allocation: its transmission
 * tables, wave batch and image accumulator live in a device array of
 * LMA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the process
 * ends (the plan's own tables, built by lma_build_basis, are read as usual). The call needs
 * ndet x probes x 8 bytes for the image, nslices x nx x ny x 8 bytes for the transmission
 * tables and at least one wave of nx x ny x 8 bytes (each rounded up to 256 bytes) within
 * that size, and returns LMA_ERR_ARG otherwise (for example the medium workload's 100 slices
 * of 512^2 do not fit; the tiny workload's 10 slices of 128^2 do). The plan's device must be
 * current. Every call on a GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (on different streams or host threads) race and must be
 * ordered by the caller. Results equal lma_plain_image's up to the order of FP64 additions. */
#define LMA_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
lma_status lma_plain_image_noalloc(lma_plan* plan, const float* potential, int32_t nslices, double* image,
                                   int32_t flags, double weight);

/* 4-D STEM output (Sec. 3.1, step 3, the pixelated detector): for every probe of the window,
 * |F(psi_p^exit)(k)|^2 / (XY) (unit incident intensity) at each of the plan's D detector
 * pixels k, the union of its rings in the order of lma_get_detector_pixels: out
 * [wh][ww][D] float32, host (the call returns when it is written) or device with
 * LMA_PTR_DEVICE. A plan whose rings include [0, a) with a at or beyond the band limit records
 * every frequency of the band. Needs a propagated basis; LMA_ERR_STATE on a partitioned plan.
 * Allocates a device buffer of the output's size for host output. */
lma_status lma_probe_patterns(lma_plan* plan, float* out, int32_t flags);

/* 3-D STEM output (Sec. 3.1, step 3, many small annuli): for every probe of the window and
 * a = 0..nbins-1, the sum of |F(psi_p^exit)(k)|^2 / (XY) over the plan's detector pixels with
 * a * width <= lambda |k| < (a + 1) * width (width in radians, 1 <= nbins <= 512): image
 * [nbins][wh][ww] float64, image = weight * I, or image += weight * I with LMA_ACCUMULATE;
 * host or device (LMA_PTR_DEVICE) as for lma_probe_image. Needs a propagated basis;
 * LMA_ERR_STATE on a partitioned plan. */
lma_status lma_probe_radial(lma_plan* plan, double width, int32_t nbins, double* image, int32_t flags,
                            double weight);

/* The plain-multislice 4-D output: every probe of the window propagated directly (Sec. 3.1
 * steps 1-3), out as for lma_probe_patterns. Does not touch the resident basis. Allocates a
 * device buffer of n_probes x D complex values for the call. */
lma_status lma_plain_patterns(lma_plan* plan, const float* potential, int32_t nslices, float* out,
                              int32_t flags);

/* Local recompute after a specimen edit (Sec. 4.2.6): re-propagate the resident translates
 * whose centre lies within radius_A of the edited pixel box, with the new potential, and
 * re-form the probes whose translate set meets them; their image values are replaced in
 * `image` (host, the layout of lma_probe_image, holding the previous image). bbox_px:
 * x0, y0, x1, y1, half-open, periodic. radius_A <= 0 selects every translate (the full
 * recompute). With translate windows (lattice.prop_nx > 0) a translate depends on the
 * potential inside its window only: a radius of half the window's diagonal makes the local
 * recompute equal to a full one. Outputs: counts of re-propagated translates and re-formed
 * probes. */
lma_status lma_recompute_local(lma_plan* plan, const float* potential_new, int32_t nslices,
                               const int32_t bbox_px[4], double radius_A, double* image,
                               int32_t* n_translates_redone, int32_t* n_probes_redone);

/* Blocks until every piece of work the plan has queued on its stream has finished. */
lma_status lma_synchronize(lma_plan* plan);

/* Picks the slice-pass schedule for an nx x ny grid by measurement: times one slice (row
 * pass, then column pass, the multislice step of Fig. multislice_pseudocode) on synthetic
 * waves for every tile width the passes are built for and every batch of 64..4096 waves
 * that fits max_bytes (0: 4 GiB), and returns the fastest. Results are kept per device and
 * grid for the life of the process; later calls return them without measuring. Allocates
 * and frees its own scratch memory; work runs on hip_stream (may be NULL) and is finished
 * on return. LMA_ERR_UNSUPPORTED for a grid the passes are not built for. */
lma_status lma_autotune(int32_t nx, int32_t ny, int64_t max_bytes, void* hip_stream, lma_tuning* out);

/* ------------------------------------------------------------------------------------------
 * Uneven batch: the translate propagation (step 1 of Fig. lma_pseudocode) of several plans,
 * of any grid sizes, slice counts and scans, as one HIP graph launch. The graph holds every
 * plan's slice loop (its passes over all its wave batches) on one of four branches; plans on
 * different branches run concurrently on the device. The graph is captured at the first
 * lma_batch_propagate and replayed afterwards.
 * ---------------------------------------------------------------------------------------- */
typedef struct lma_batch lma_batch;

/* plans[n]: device plans on the current device, none partitioned, each at most once;
 * nslices[n] >= 1 slices per plan. hip_stream: the stream the graph is launched on (NULL:
 * the batch creates its own). Reserves each plan's transmission tables for its nslices. The
 * plans must outlive the batch. */
lma_status lma_batch_create(lma_plan* const* plans, int32_t n, const int32_t* nslices, void* hip_stream,
                            lma_batch** out);
/* potentials[n]: [nslices[i]][ny_i][nx_i] each (device pointers with LMA_PTR_DEVICE, else
 * host; host ones are read before the call returns). Forms every plan's transmission tables
 * on the plan's stream, then launches the graph; afterwards each plan's stream is ordered
 * after the graph, so lma_probe_image on a plan sees its new basis. With host potentials the
 * call returns when the propagation has finished. */
lma_status lma_batch_propagate(lma_batch* batch, const float* const* potentials, int32_t flags);
void lma_batch_destroy(lma_batch* batch);
/* The same batch with plans of one transform-length class sharing their passes (the uneven
 * batch's persistent launches per length class; the multislice step of Fig.
 * multislice_pseudocode): plans with the same grid, tile width and band gap, bitwise the same
 * propagator table and no translate windows hold all their translate waves in one device
 * buffer of at most max_group_bytes (0: 32 GiB; a class that needs more is split), and each
 * slice's row pass (every wave multiplied by its own plan's t_j) and column pass are one
 * persistent launch over all of that buffer's waves still propagating; each plan's initial
 * waves and its last column pass (the gather into its basis) stay its own. Other plans run
 * their own slice loop as in lma_batch_create. Groups and those plans are spread over the
 * graph's four branches. Same arguments and use otherwise; LMA_ERR_OOM when a group buffer
 * cannot be allocated (nothing is kept). */
lma_status lma_batch_create_grouped(lma_plan* const* plans, int32_t n, const int32_t* nslices, void* hip_stream,
                                    int64_t max_group_bytes, lma_batch** out);

/* Device bytes a plan with these arguments would hold for nslices slices: the memory side of
 * the translate reuse of Sec. 4.2.4 (every propagated translate the window needs kept
 * resident, |rows| x D x 8 bytes, which the paper's partition strategies trade against
 * multislice runs), plus the wave batch (batch x X x Y x 8 bytes), the nslices transmission
 * tables and potential staging (12 bytes per pixel each), the window's image and the plan's
 * tables, counted term by term from the host plan (an upper estimate of what lma_build_basis
 * and lma_propagate allocate for that slice count; the figure the server admits a specimen
 * by). Nothing is allocated (host planning only); *bytes is written on success. LMA_ERR_ARG for a null bytes, nslices < 1 or
 * arguments lma_build_basis would refuse; LMA_ERR_OOM when host planning runs out of memory. */
lma_status lma_footprint(const lma_optics* optics, const lma_lattice* lattice,
                         const lma_detectors* detectors, int32_t nslices, int64_t* bytes);

/* ------------------------------------------------------------------------------------------
 * Serving: a request loop with continuous batching over resident specimens.
 *
 * A server holds up to max_specimens resident plans (specimens), each on its own stream, and
 * runs requests on `slots` worker threads. Requests of one specimen run one at a time in
 * submission order; requests of different specimens run concurrently, so work that arrives
 * while others are on the GPU starts as soon as a slot is free and overlaps on the device.
 * Building a specimen is admitted by its device footprint (lma_footprint for the request's
 * nslices) against budget_bytes; builds are admitted in submission order and wait until
 * released specimens free enough memory. Latency is measured from submission to completion
 * of the request's device work.
 * ---------------------------------------------------------------------------------------- */
typedef struct lma_server lma_server;

enum {
  LMA_REQ_BUILD = 1,    /* lma_build_basis (own stream) for `specimen`                     */
  LMA_REQ_IMAGE = 2,    /* lma_image: the specimen's LMA image for a potential              */
  LMA_REQ_EDIT = 3,     /* lma_recompute_local after a local edit (host image, patched)     */
  LMA_REQ_PLAIN = 4,    /* lma_plain_image: plain multislice image of the specimen's window */
  LMA_REQ_RELEASE = 5   /* lma_destroy: frees the specimen's device memory                  */
};

typedef struct {
  int32_t kind;                    /* LMA_REQ_*                                             */
  int32_t specimen;                /* 0 <= specimen < max_specimens                         */
  const lma_optics* optics;        /* BUILD: copied at submission                           */
  const lma_lattice* lattice;      /* BUILD: copied at submission                           */
  const lma_detectors* detectors;  /* BUILD: copied at submission (ring arrays too)         */
  const float* potential;          /* IMAGE, PLAIN, EDIT: [nslices][ny][nx]; the caller    */
                                   /* keeps it valid until the request has completed       */
  int32_t nslices;                 /* IMAGE, PLAIN, EDIT; BUILD: slices the footprint holds */
  double* image;                   /* IMAGE, PLAIN: [n_det][h][w] (host, or device with    */
                                   /* LMA_PTR_DEVICE); EDIT: host image patched in place   */
  int32_t flags;                   /* IMAGE, PLAIN: LMA_PTR_DEVICE, LMA_ACCUMULATE; BUILD:  */
                                   /* LMA_HOST_ONLY plans on the host only (no device work; */
                                   /* the specimen then answers IMAGE, PLAIN and EDIT with  */
                                   /* LMA_ERR_STATE)                                         */
  double weight;                   /* IMAGE, PLAIN                                          */
  int32_t bbox[4];                 /* EDIT: edited pixels x0, y0, x1, y1 (half-open)        */
  double radius;                   /* EDIT: recompute radius, Angstrom                      */
} lma_request;

/* slots >= 1 worker threads, 1 <= max_specimens <= 4096, budget_bytes > 0. */
lma_status lma_server_create(int32_t slots, int32_t max_specimens, int64_t budget_bytes, lma_server** out);
/* Queues a request (arguments checked here) and returns its ticket (>= 1). LMA_ERR_ARG for a
 * malformed request; the status of the work itself is reported by lma_server_wait. */
lma_status lma_server_submit(lma_server* server, const lma_request* request, int64_t* ticket);
/* Blocks until the ticket's request has completed and returns its status (the call's own
 * lma_status, with its message in lma_last_error); latency_ms (submission to completion) and
 * service_ms (start to completion) may be NULL. Each ticket can be waited for once: a ticket
 * never issued, or already waited for, returns LMA_ERR_ARG at once. A BUILD for a specimen
 * that is resident when it runs fails with LMA_ERR_STATE and leaves the specimen and the
 * admitted bytes as they were. */
lma_status lma_server_wait(lma_server* server, int64_t ticket, double* latency_ms, double* service_ms);
/* The specimen's resident plan (NULL if none); valid until a RELEASE of it completes. */
lma_status lma_server_plan(lma_server* server, int32_t specimen, lma_plan** plan);
/* Device bytes admitted (footprints of resident and building specimens). */
lma_status lma_server_in_use(lma_server* server, int64_t* bytes);
/* Runs every queued request, stops the workers and destroys the resident plans. */
void lma_server_destroy(lma_server* server);

/* Inspection (host logic; work on host-only plans). Arrays are caller-allocated with the
 * sizes given by lma_plan_info. */
lma_status lma_plan_info(const lma_plan* plan, lma_info* out);
/* I_f positions, double [n_translates][2], Angstrom, translate t = b*Rfx + a. */
lma_status lma_get_translates(const lma_plan* plan, double* pos);
/* Per coefficient set s (s = sy*ncls_x + sx): translate indices of its L nearest
 * translates (int32 [n_sets][L]) and their coefficients (double [n_sets][L][2]). */
lma_status lma_get_coefficients(const lma_plan* plan, int32_t* translate, double* alpha);
/* Detector pixels: flat index ky*nx + kx (int32 [D]) and ring bit mask (uint32 [D]). */
lma_status lma_get_detector_pixels(const lma_plan* plan, int32_t* flat, uint32_t* mask);
/* Normalised probe spectrum psi_0-hat (sum |.|^2 = XY), double [ny][nx][2]. */
lma_status lma_get_probe_spectrum(const lma_plan* plan, double* spec);
/* Normalised spectrum of the input wave u (sum |.|^2 = XY), double [ny][nx][2]. */
lma_status lma_get_input_wave_spectrum(const lma_plan* plan, double* spec);
/* With translate windows (lattice.prop_nx > 0): the window DFT of u cropped to a window
 * centred on it, double [prop_ny][prop_nx][2]; LMA_ERR_STATE without windows. */
lma_status lma_get_window_spectrum(const lma_plan* plan, double* spec);
/* The resident basis (the propagated translates kept for reuse, Sec. 4.2.4) written to a file
 * and read back, so that a specimen's propagation outlives the process that computed it.
 * The file holds a header and the rows in the device's encoding; its fingerprint covers the
 * optics, the input wave and translate lattice, the element encoding, the translate windows,
 * the detector pixels and the resident translates (not the potential, which the caller
 * pairs with the file). lma_save_basis needs a valid basis; lma_load_basis checks the header
 * and the file's length against the plan before it copies anything to the device
 * (LMA_ERR_ARG, basis unchanged, on a mismatch) and leaves the basis valid on success.
 * Both stream through 64 MiB of host memory and synchronise the plan's stream.
 * LMA_ERR_STATE on host-only and partitioned plans. */
lma_status lma_save_basis(lma_plan* plan, const char* path);
lma_status lma_load_basis(lma_plan* plan, const char* path);

/* Resident-basis rows first..first+count-1 (rows in increasing translate order, see
 * lma_get_rows): F(U_i) at the D detector pixels, float [count][D][2] on the host. */
lma_status lma_get_basis_rows(lma_plan* plan, int32_t first, int32_t count, float* out);
/* Translate index of each resident row, int32 [n_rows]. */
lma_status lma_get_rows(const lma_plan* plan, int32_t* translate);

/* Kernel timing with hipEvents around every launch (adds a little overhead). */
lma_status lma_set_timing(lma_plan* plan, int32_t enable);
/* Fills up to max entries, returns the count in *n; resets the counters if reset != 0. */
lma_status lma_get_timing(lma_plan* plan, lma_kernel_time* out, int32_t max, int32_t* n,
                          int32_t reset);

void lma_destroy(lma_plan* plan);
const char* lma_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LMA_H */

"""Benchmark: STEM pixels/s of the LMA hot path against plain multislice on one MI355X.

One step = one frozen-phonon configuration of the medium workload pushed through the whole
hot path: lma_propagate (initial translates, 100 x [row pass: row IFFT, transmission, row FFT;
column pass: column FFT, propagator, column IFFT], exit spectra kept at the detector pixels)
then lma_probe_image (coefficient contraction and detector rings, accumulated with weight
1/n_phonons). The plain multislice comparator (lma_plain_image) runs the same configurations.
Potentials of every configuration are resident in HBM before the timed region.

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "medium"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2310_16829_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic_medium.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# ------------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the same workload
# ------------------------------------------------------------------------------------------
def _oracle_wave(args):
    import numpy as np
    from oracle.lma import translate_wave
    from oracle.multislice import multislice
    pos = args
    st, v = _oracle_wave.st, _oracle_wave.v
    u0 = translate_wave(st, st.spec0, pos)
    return np.fft.fft2(multislice(u0, v, st.sigma, st.prop))


def _oracle_init(spec):
    from oracle import physics as ph
    from oracle.multislice import Setup
    from synth import WORKLOADS, potential_slices
    w = WORKLOADS[spec]
    _oracle_wave.v = potential_slices(w, 0)
    _oracle_wave.st = Setup(w.nx, w.ny, w.lx, w.ly, ph.electron_wavelength(w.kv), ph.interaction_constant(w.kv),
                            w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs, w.scan,
                            [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors])


BASELINE_PROBE = (37, 101)       # the medium workload's probe whose LMA pixel the oracle forms


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_translates, n_probes, plan, images):
    """Times the oracle on a sample and scales to one full image of one phonon configuration,
    T = |I_f| t_wave + |P| t_probe. The sample is one probe's LMA pixel: its L nearest translates
    propagated by the FP64 oracle in parallel (one process per core), then their combination
    with the oracle's own least-squares coefficients and the detector sums. With `plan` holding
    the FP32 basis of phonon configuration 0, the same run states the GPU's error against the
    oracle: every sampled translate's exit wave at the detector pixels, and the LMA pixel of
    `images` ({name: [n_det][Py][Px] image of configuration 0}) per detector."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    from oracle import physics as ph
    from oracle.lma import Lattice, least_squares
    affinity = len(os.sched_getaffinity(0))
    # one GPU's share of the host: 16 cores (the process count this machine allows per GPU)
    cores = max(1, min(16, affinity))
    if not hasattr(_oracle_wave, "st"):
        _oracle_init(WORKLOAD)
    st = _oracle_wave.st
    R = (w.nx // w.basis_px, w.ny // w.basis_px)
    ol = Lattice(st, R, 1, w.offset_frac, w.L)
    nbr = ol.nearest(*BASELINE_PROBE)
    positions = [tuple(float(c) for c in ol.translate_position(ta, tb)) for ta, tb in nbr]
    with ProcessPoolExecutor(cores, initializer=_oracle_init, initargs=(WORKLOAD,)) as ex:
        list(ex.map(_oracle_wave, positions[:cores]))          # start-up and potential generation
        t0 = time.perf_counter()
        spectra = list(ex.map(_oracle_wave, positions))
        t_waves = time.perf_counter() - t0
    t_wave = t_waves / len(positions)                          # wall time per wave at `cores` workers
    alpha, _, resid = least_squares(st, ol, st.spec0, *BASELINE_PROBE)
    t0 = time.perf_counter()
    spec = np.zeros_like(spectra[0])
    for c, sp in zip(alpha, spectra):
        spec += c * sp
    ref = ph.detector_values(spec, st.masks)
    t_probe = (time.perf_counter() - t0) / cores                # probes spread over the same cores
    t_image = n_translates * t_wave + n_probes * t_probe
    t_plain = n_probes * t_wave
    flat, _ = plan.detector_pixels()
    rows = plan.rows()
    row_of = {int(t): r for r, t in enumerate(rows)}
    wave_err = []
    for (ta, tb), sp in zip(nbr, spectra):
        got = plan.basis_rows(row_of[tb * ol.Rfx + ta], 1)[0]
        ref_w = sp.ravel()[flat]
        wave_err.append(float(np.linalg.norm(got - ref_w) / np.linalg.norm(ref_w)))
    a, b = BASELINE_PROBE
    pixel_err = {name: [float(abs(img[r, b, a] - ref[r]) / abs(ref[r])) for r in range(len(ref))]
                 for name, img in images.items()}
    return {
        "value": n_probes / t_image, "unit": "STEM pixels/s", "cores": cores, "kind": "oracle",
        "cpu_model": cpu_model(), "cores_in_affinity": affinity,
        "plain_value": n_probes / t_plain,
        "sample": (f"the LMA pixel of probe {BASELINE_PROBE} of the medium workload: its {len(positions)} nearest "
                   f"translates (512^2, 100 slices) propagated by the FP64 oracle on {cores} processes "
                   f"({t_wave:.3f} s wall per wave), combined with the oracle's least-squares coefficients "
                   f"({t_probe * cores:.3f} s); scaled to one phonon image: {n_translates} translates + "
                   f"{n_probes} probes"),
        "error_vs_oracle": {
            "exit_wave_rel_l2_max": max(wave_err), "exit_wave_rel_l2_median": float(np.median(wave_err)),
            "translates": len(wave_err), "lma_pixel": list(BASELINE_PROBE),
            "lma_pixel_rel_err_per_detector": pixel_err, "probe_lsq_residual": float(resid),
            "what": "GPU exit waves (FP32) at the detector pixels and the LMA pixel's detector values against the "
                    "FP64 oracle, phonon configuration 0"},
    }


def spacing_study(w):
    """Speed and LMA-vs-plain error of the medium workload (configuration 0) at translate
    spacings of 4, 8 and 16 px (0.4, 0.8, 1.6 A; the probe needs <= lambda/(2 alpha) = 0.63 A)."""
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth import potential_slices
    v = torch.from_numpy(potential_slices(w, 0)).cuda()
    lam, sig = lma.electron_constants(w.kv)
    rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
    opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)

    def run(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    base = lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], 128, 128, 1, (0.5, 0.5), w.L), lma.detectors(rings))
    plain, t_plain = run(lambda: base.plain_image(v, device=True))
    plain = plain.cpu().numpy()
    base.close()
    rows = []
    for spacing_px, L in ((4, 144), (8, 144), (16, 148)):
        R = w.nx // spacing_px
        plan = lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], R, R, 1, (0.5, 0.5), L), lma.detectors(rings))

        def step():
            plan.propagate(v)
            return plan.probe_image(device=True)
        img, t = run(step)
        img = img.cpu().numpy()
        err = [float(np.linalg.norm(img[r] - plain[r]) / np.linalg.norm(plain[r])) for r in range(len(rings))]
        rows.append({"spacing_px": spacing_px, "spacing_A": spacing_px * w.lx / w.nx, "L": L,
                     "translates": plan.info().n_rows, "probe_residual": plan.info().max_residual,
                     "seconds": t, "speedup_vs_plain": t_plain / t,
                     "lma_vs_plain_rel_l2": dict(zip([d[0] for d in w.detectors], err))})
        plan.close()
    print(json.dumps({"study": "translate spacing, medium workload, configuration 0", "plain_seconds": t_plain,
                      "rows": rows}), flush=True)


def window_study(w):
    """Option (ii): the medium workload (configuration 0, translates every 4 px, L = 144) with
    every translate propagated on a window of 64, 128 or 256 pixels centred on it, and on the
    whole cell: LMA time (propagation + contraction), speed-up
    over plain multislice of the whole cell, and the LMA-vs-plain image error per detector."""
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth import potential_slices
    v = torch.from_numpy(potential_slices(w, 0)).cuda()
    lam, sig = lma.electron_constants(w.kv)
    rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
    opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)

    def run(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    base = lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], 128, 128, 1, (0.5, 0.5), w.L), lma.detectors(rings))
    plain, t_plain = run(lambda: base.plain_image(v, device=True))
    plain = plain.cpu().numpy()
    base.close()
    rows = []
    for side in (64, 128, 256, 0):
        plan = lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], 128, 128, 1, (0.5, 0.5), w.L, prop_window=(side, side)),
                        lma.detectors(rings))

        def step():
            plan.propagate(v)
            return plan.probe_image(device=True)
        img, t = run(step)
        img = img.cpu().numpy()
        err = [float(np.linalg.norm(img[r] - plain[r]) / np.linalg.norm(plain[r])) for r in range(len(rings))]
        rows.append({"window_px": side or w.nx, "window_A": (side or w.nx) * w.lx / w.nx, "seconds": t,
                     "speedup_vs_plain": t_plain / t,
                     "lma_vs_plain_rel_l2": dict(zip([d[0] for d in w.detectors], err))})
        log(f"window {side or w.nx}: {t:.3f} s, errors {err}")
        plan.close()
    print(json.dumps({"study": "translate windows (option (ii)), medium workload, configuration 0",
                      "plain_seconds": t_plain, "rows": rows}), flush=True)


# ------------------------------------------------------------------------------------------
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense

KERNEL_NAMES = (("k_contract_bf16", "contract_bf16"), ("k_contract_mfma2_dma", "contract_mfma"), ("k_contract_mfma2", "contract_mfma"), ("k_contract_mfma", "contract_mfma"), ("k_contract", "contract"),
                ("k_transmission", "transmission"), ("k_scale_out", "scale_out"), ("k_embed", "embed"),
                ("k_intensity", "intensity"))
PASS_MODES = {"0": "row_pass", "1": "col_pass", "2": "init", "3": "col_gather", "4": "col_reduce", "5": "row_pass",
              "6": "row_pass"}


def _short_name(kernel: str):
    import re
    m = re.search(r"k_pass<\d+, \d+, (\d)(?:, \d+)*>", kernel)
    if m:
        return PASS_MODES.get(m.group(1))
    for tag, name in KERNEL_NAMES:
        if tag + "<" in kernel or tag + "(" in kernel:
            return name
    if "copyBuffer" in kernel:
        return "copy"
    return None


def _counter_means(run_dir: str, counter: str):
    """Mean per dispatch of one rocprofv3 counter (KiB for FETCH_SIZE / WRITE_SIZE), by kernel."""
    import csv
    import glob
    per = {}
    for path in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                name = _short_name(r["Kernel_Name"])
                if name is None:
                    continue
                d = per.setdefault(name, {})
                d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in per.items()}


def summarize_counters(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir):
    """HBM bytes per launch of every kernel from FETCH_SIZE and WRITE_SIZE runs, each scaled by
    what the same counter reads for a 1 GiB device copy (bench.py --copy-calibration)."""
    copy_bytes = 1 << 30
    cf = _counter_means(cal_fetch_dir, "FETCH_SIZE")["copy"][1]
    cw = _counter_means(cal_write_dir, "WRITE_SIZE")["copy"][1]
    ff, wf = copy_bytes / 1024 / cf, copy_bytes / 1024 / cw
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        kernels[k] = {"dispatches": fetch[k][0], "FETCH_SIZE_KiB": fetch[k][1], "WRITE_SIZE_KiB": write[k][1],
                      "hbm_bytes_per_launch": (fetch[k][1] * ff + write[k][1] * wf) * 1024}
    print(json.dumps({"kernel_source_hash": kernel_source_hash(), "workload": WORKLOAD,
                      "calibration": {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB": cf, "WRITE_SIZE_KiB": cw,
                                      "fetch_factor": ff, "write_factor": wf},
                      "kernels": kernels}, indent=1))


def summarize_pmc(run_dirs, n_cu=256):
    """Per-kernel means per dispatch of every counter in rocprofv3 --pmc runs, with the
    utilisations they give. SQ_BUSY_CU_CYCLES sums busy cycles over the CUs (256 x the kernel's
    duration x 2.4 GHz, within a few percent); per SIMD: MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES /
    (SQ_BUSY_CU_CYCLES x 4 SIMDs); VALU issue = SQ_INSTS_VALU x 4 cycles (a 64-wide wavefront
    on a 16-lane SIMD) / (SQ_BUSY_CU_CYCLES x 4 SIMDs); MFMA flops = MOPS x 512."""
    import csv
    import glob
    per = {}
    for d in run_dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    name = _short_name(r["Kernel_Name"])
                    if name is None:
                        continue
                    c = per.setdefault(name, {}).setdefault(r["Counter_Name"], {})
                    c[r["Dispatch_Id"]] = c.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    out = {}
    for k, cs in sorted(per.items()):
        m = {c: sum(v.values()) / len(v) for c, v in cs.items()}
        m["dispatches"] = max(len(v) for v in cs.values())
        if "SQ_BUSY_CU_CYCLES" in m:
            m["busy_us"] = m["SQ_BUSY_CU_CYCLES"] / n_cu / 2.4e3
            if "SQ_VALU_MFMA_BUSY_CYCLES" in m:
                m["mfma_busy"] = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (m["SQ_BUSY_CU_CYCLES"] * 4)
            if "SQ_INSTS_VALU" in m:
                m["valu_issue"] = m["SQ_INSTS_VALU"] * 4 / (m["SQ_BUSY_CU_CYCLES"] * 4)
        for dt in ("F32", "BF16"):
            if f"SQ_INSTS_VALU_MFMA_MOPS_{dt}" in m:
                m[f"mfma_tflop_{dt.lower()}"] = m[f"SQ_INSTS_VALU_MFMA_MOPS_{dt}"] * 512 / 1e12
        out[k] = m
    print(json.dumps({"kernel_source_hash": kernel_source_hash(), "workload": WORKLOAD, "kernels": out}, indent=1))


def serve(rates=(2.0, 10.0, 50.0, 200.0), n_requests=60, slots=4, emit=True, cap_seconds=8.0):
    """Serving under Poisson arrivals, once with FP32 basis rows and contraction and once with
    the basis stored as split BF16 (hi + lo): see serve_mode."""
    import paper_2310_16829_amd as lma
    out = {"study": "serving: Poisson arrivals over 6 resident specimens (2 x 128^2 x 10 slices, 2 x 256^2 x 20 "
                    "slices, 2 x the medium 512^2 x 100-slice specimen on 16 x 16-probe windows), 70 % LMA "
                    "images, 30 % local edits", "slots": slots}
    for name, prec in (("fp32", lma.LMA_GEMM_FP32), ("split_bf16", lma.LMA_GEMM_SPLIT_BF16)):
        log(f"serve: {name}")
        out[name] = serve_mode(prec, rates, n_requests, slots, cap_seconds)
    if emit:
        print(json.dumps(out), flush=True)
    return out


def serve_mode(precision, rates, n_requests, slots, cap_seconds=8.0):
    """Six resident specimens of mixed sizes (128^2 x 10 slices, 256^2 x 20 slices, the 512^2 x
    100-slice medium specimen on a 16 x 16-probe window), 70 % image requests (a new
    frozen-phonon configuration of a random specimen) and 30 % local edits (one raised 12 x
    12-pixel column patch of a random specimen, recomputed locally), run by the library's
    request loop with `slots` worker slots. Returns p50 / p99 latency (arrival to completion)
    and throughput per arrival rate."""
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth import WORKLOADS, potential_slices

    rng = np.random.default_rng(2024)
    wt, wm = WORKLOADS["tiny"], WORKLOADS["medium"]
    lam, sig = lma.electron_constants(200.0)
    rings = [(a * 1e-3, b * 1e-3) for _, a, b in wt.detectors[1:]]
    specs = []
    for n, nsl, kind in ((128, 10, "tiny"), (128, 10, "tiny"), (256, 20, "mid"), (256, 20, "mid"),
                         (512, 100, "medium"), (512, 100, "medium")):
        l = n * 0.1
        opt = lma.optics(n, n, l, l, lam, sig, 2.0, 2.0 / 3.0, 0.02)
        if kind == "medium":
            a0, b0 = (int(x) for x in rng.integers(0, 112, size=2))
            lat = lma.lattice(128, 128, 128, 128, 1, (0.5, 0.5), 144, precision, window=(a0, b0, 16, 16))
            pots = [potential_slices(wm, c) for c in range(2)]
        else:
            lat = lma.lattice(n // 8, n // 8, n // 4, n // 4, 1, (0.5, 0.5), 36, precision)
            pots = [rng.uniform(0, 40, size=(nsl, n, n)).astype(np.float32) for _ in range(2)]
        shape = (len(rings), lat.window[3] or lat.py, lat.window[2] or lat.px)
        specs.append(dict(opt=opt, lat=lat, det=lma.detectors(rings), pots=[torch.from_numpy(v).cuda() for v in pots],
                          host=pots[0], n=n, shape=shape, kind=kind))
    torch.cuda.synchronize()
    budget = 64 << 30
    out = {"rates": []}
    with lma.Server(slots, len(specs), budget) as srv:
        t = [srv.build(k, s["opt"], s["lat"], s["det"], s["pots"][0].shape[0]) for k, s in enumerate(specs)]
        for x in t:
            srv.wait(x)
        for k, s in enumerate(specs):
            srv.wait(srv.image(k, s["pots"][0], torch.zeros(s["shape"], dtype=torch.float64, device="cuda")))
        out["resident_bytes"] = srv.in_use()
        for rate in rates:
            # about cap_seconds of arrivals at most (all n_requests without a cap)
            n_req = n_requests if cap_seconds is None else max(16, min(n_requests, int(rate * cap_seconds)))
            gaps = rng.exponential(1.0 / rate, size=n_req)
            reqs = []
            for i in range(n_req):
                k = int(rng.integers(0, len(specs)))
                if rng.random() < 0.3:
                    s = specs[k]
                    v = s["host"].copy()
                    x0, y0 = (int(q) for q in rng.integers(0, s["n"] - 12, size=2))
                    v[:, y0:y0 + 12, x0:x0 + 12] += 15.0
                    reqs.append(("edit", k, v, (x0, y0, x0 + 12, y0 + 12)))
                else:
                    reqs.append(("image", k, int(rng.integers(0, 2)), None))
            torch.cuda.synchronize()
            tickets = []
            t0 = time.monotonic()
            arrival = t0
            for (kind, k, arg, bbox), gap in zip(reqs, gaps):
                arrival += gap
                delay = arrival - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
                s = specs[k]
                if kind == "edit":
                    tickets.append((kind, srv.edit(k, arg, bbox, 2.0, np.zeros(s["shape"]))))
                else:
                    img = torch.empty(s["shape"], dtype=torch.float64, device="cuda")
                    tickets.append((kind, srv.image(k, s["pots"][arg], img)))
            lat = {"image": [], "edit": []}
            svc = []
            for kind, tk in tickets:
                l, sv = srv.wait(tk)
                lat[kind].append(l)
                svc.append(sv)
            wall = time.monotonic() - t0
            allv = lat["image"] + lat["edit"]
            row = {"rate_per_s": rate, "requests": n_req, "throughput_per_s": n_req / wall,
                   "p50_ms": float(np.percentile(allv, 50)), "p99_ms": float(np.percentile(allv, 99)),
                   "image_p50_ms": float(np.percentile(lat["image"], 50)) if lat["image"] else None,
                   "image_p99_ms": float(np.percentile(lat["image"], 99)) if lat["image"] else None,
                   "edit_p50_ms": float(np.percentile(lat["edit"], 50)) if lat["edit"] else None,
                   "edit_p99_ms": float(np.percentile(lat["edit"], 99)) if lat["edit"] else None,
                   "mean_service_ms": float(np.mean(svc))}
            log(f"serve: rate {rate}/s: p50 {row['p50_ms']:.1f} ms, p99 {row['p99_ms']:.1f} ms, "
                f"{row['throughput_per_s']:.1f} req/s")
            out["rates"].append(row)
    return out


def _edit_potential(w, base, c, col_xy, seed):
    """The potential of workload w (configuration c, whose potential is `base`) after one local
    edit of the generator (one atomic column: a new species amplitude, each of its atoms kept
    with probability 1/2), and the edited pixel box: base minus the column's old Gaussians plus
    its new ones (the column: the atoms within 1 A of its site in x, y; the nearest other
    column is 2.9 A away)."""
    import numpy as np
    from synth.specimen import atom_sites, edit_column, phonon_positions, potential_from_atoms
    sites, amps0 = atom_sites(w)
    pos0 = phonon_positions(w, c, sites)
    pos1, amps1, bbox = edit_column(w, c, col_xy, seed=seed)
    d2 = (sites[:, 0] - col_xy[0]) ** 2 + (sites[:, 1] - col_xy[1]) ** 2
    centres = np.unique(sites[d2 <= d2.min() + 1e-9][:, :2], axis=0)   # the edited column(s)

    def column(pos):
        hit = np.zeros(len(pos), dtype=bool)
        for cx, cy in centres:
            dx = pos[:, 0] - cx
            dx -= w.lx * np.round(dx / w.lx)
            dy = pos[:, 1] - cy
            dy -= w.ly * np.round(dy / w.ly)
            hit |= dx * dx + dy * dy < 1.0
        return hit
    c0, c1 = column(pos0), column(pos1)
    v = base.copy()
    v += potential_from_atoms(w, pos1[c1], amps1[c1])
    v -= potential_from_atoms(w, pos0[c0], amps0[c0])
    return v, bbox


def serve_c5(precision, rates, n_requests=200, slots=4):
    """The serving workload drawn from the sizes of the other workloads: the tiny specimen (128^2,
    10 slices, its full 16 x 16 scan), the medium one (512^2, 100 slices) on a 16 x 16-probe
    window, the large one (2048^2, 250 slices, 300 kV) on a 16 x 16-probe sub-scan, and one
    specimen of every side of the uneven batch (96 ... 640 px, 20-200 slices) on a window of up
    to 16 x 16 probes. Requests: 70 % LMA images of a frozen-phonon configuration, 30 % local
    edits that replace one atomic column (species amplitude and occupancy) and recompute the
    affected translates; a specimen is drawn with weight 1, the large one with weight 0.2 (an
    image of its sub-scan is ~15 s of device time). Poisson arrivals, n_requests per rate."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth import WORKLOADS, potential_slices
    from synth.specimen import uneven_batch

    rng = np.random.default_rng(5)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    ws = [WORKLOADS["tiny"], WORKLOADS["medium"], WORKLOADS["large"]]
    seen = set()
    for w in uneven_batch(64):
        if w.nx not in seen:
            seen.add(w.nx)
            ws.append(w)
    specs = []
    for w in ws:
        big = w.name == "large"
        log(f"serve c5: specimen {w.name} ({w.nx}^2 x {w.nslices} slices)")
        lam, sig = lma.electron_constants(w.kv)
        rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
        opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)
        (Rx, Ry), f = w.lattice_size()
        side = max(2, min(16, w.scan[0], (16 * w.scan[0]) // Rx))
        a0 = int(rng.integers(0, w.scan[0] - side + 1))
        b0 = int(rng.integers(0, w.scan[1] - side + 1))
        lat = lma.lattice(w.scan[0], w.scan[1], Rx, Ry, f, w.offset_frac, w.L, precision, window=(a0, b0, side, side))
        n_cfg = 1 if big else 2
        if big:
            step = -(-w.nslices // cores)
            with ProcessPoolExecutor(cores) as ex:
                pots = [np.concatenate(list(ex.map(_large_slices, [(lo, min(lo + step, w.nslices))
                                                                   for lo in range(0, w.nslices, step)])))]
        else:
            pots = [potential_slices(w, c) for c in range(n_cfg)]
        # edited potentials: columns near the window's centre
        cx = (a0 + side / 2) * w.lx / w.scan[0]
        cy = (b0 + side / 2) * w.ly / w.scan[1]
        n_edits = 1 if big else 2
        edits = [_edit_potential(w, pots[0], 0, (cx + 2.0 * e, cy - 1.5 * e), e) for e in range(n_edits)]
        specs.append(dict(w=w, opt=opt, lat=lat, det=lma.detectors(rings), weight=0.2 if big else 1.0,
                          pots=[torch.from_numpy(v).cuda() for v in pots], edits=edits,
                          shape=(len(rings), side, side)))
        del pots
    torch.cuda.synchronize()
    weights = np.array([s["weight"] for s in specs])
    weights /= weights.sum()
    out = {"study": "serving, config-5 mix: " + ", ".join(f"{s['w'].name} {s['w'].nx}^2x{s['w'].nslices}" for s in specs),
           "precision": "split_bf16" if precision == lma.LMA_GEMM_SPLIT_BF16 else "fp32", "slots": slots,
           "rates": []}
    with lma.Server(slots, len(specs), 200 << 30) as srv:
        t = [srv.build(k, s["opt"], s["lat"], s["det"], s["w"].nslices) for k, s in enumerate(specs)]
        for x in t:
            srv.wait(x)
        for k, s in enumerate(specs):
            srv.wait(srv.image(k, s["pots"][0], torch.zeros(s["shape"], dtype=torch.float64, device="cuda")))
        out["resident_bytes"] = srv.in_use()
        for rate in rates:
            gaps = rng.exponential(1.0 / rate, size=n_requests)
            reqs = []
            for i in range(n_requests):
                k = int(rng.choice(len(specs), p=weights))
                s = specs[k]
                if rng.random() < 0.3:
                    reqs.append(("edit", k, int(rng.integers(0, len(s["edits"])))))
                else:
                    reqs.append(("image", k, int(rng.integers(0, len(s["pots"])))))
            torch.cuda.synchronize()
            tickets = []
            t0 = time.monotonic()
            arrival = t0
            for (kind, k, arg), gap in zip(reqs, gaps):
                arrival += gap
                delay = arrival - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
                s = specs[k]
                if kind == "edit":
                    v, bbox = s["edits"][arg]
                    tickets.append((kind, k, srv.edit(k, v, bbox, 2.5, np.zeros(s["shape"]))))
                else:
                    img = torch.empty(s["shape"], dtype=torch.float64, device="cuda")
                    tickets.append((kind, k, srv.image(k, s["pots"][arg], img)))
            lat = {"image": [], "edit": []}
            per_spec = {}
            for kind, k, tk in tickets:
                l, _ = srv.wait(tk)
                lat[kind].append(l)
                per_spec.setdefault(specs[k]["w"].name, []).append(l)
            wall = time.monotonic() - t0
            allv = lat["image"] + lat["edit"]
            row = {"rate_per_s": rate, "requests": n_requests, "throughput_per_s": n_requests / wall,
                   "p50_ms": float(np.percentile(allv, 50)), "p99_ms": float(np.percentile(allv, 99)),
                   "image_p50_ms": float(np.percentile(lat["image"], 50)) if lat["image"] else None,
                   "image_p99_ms": float(np.percentile(lat["image"], 99)) if lat["image"] else None,
                   "edit_p50_ms": float(np.percentile(lat["edit"], 50)) if lat["edit"] else None,
                   "edit_p99_ms": float(np.percentile(lat["edit"], 99)) if lat["edit"] else None,
                   "p50_ms_by_specimen": {n: float(np.percentile(v, 50)) for n, v in per_spec.items()},
                   "requests_by_specimen": {n: len(v) for n, v in per_spec.items()}}
            log(f"serve c5: rate {rate}/s: p50 {row['p50_ms']:.1f} ms, p99 {row['p99_ms']:.1f} ms, "
                f"{row['throughput_per_s']:.1f} req/s")
            out["rates"].append(row)
    return out


def paper_shaped(emit=True):
    """The paper's local-edit experiment in shape (1024^2 px over 84.536 x 79.941 A, scan
    424 x 400, I = P + p/2, f = 2, L = 59, 200 kV, 26 mrad, Z = 100 A, C_s = -2000 A) with the
    synthetic FCC specimen, 50 slices, one phonon configuration: the full LMA image (42400
    propagated translates for 169600 probes), plain multislice timed on a 64 x 64-probe window
    of the same scan (its pixel rate does not depend on the window), and the LMA-vs-plain
    image error on that window."""
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth import WORKLOADS, potential_slices

    w = WORKLOADS["paper"]
    v = torch.from_numpy(potential_slices(w, 0)).cuda()
    lam, sig = lma.electron_constants(w.kv)
    rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
    opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)
    (Rx, Ry), f = w.lattice_size()
    det = lma.detectors(rings)
    win = (180, 168, 64, 64)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    # the same kernels once on a small window first (first-launch costs out of the timings)
    with lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], Rx, Ry, f, w.offset_frac, w.L, window=(0, 0, 8, 8)), det) as p:
        p.propagate(v)
        p.probe_image()
        p.plain_image(v, device=True)
    log("paper-shaped: LMA plan (full scan)")
    plan = lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], Rx, Ry, f, w.offset_frac, w.L), det)
    info = plan.info()
    img = torch.zeros(plan.image_shape(), dtype=torch.float64, device="cuda")
    _, t_prop = timed(lambda: plan.propagate(v))
    _, t_img = timed(lambda: plan.probe_image(img))
    t_lma = t_prop + t_img
    log(f"paper-shaped: LMA {t_lma:.2f} s ({t_prop:.2f} s propagation, {t_img:.3f} s contraction)")
    lma_win = img.cpu().numpy()[:, win[1]:win[1] + win[3], win[0]:win[0] + win[2]]
    plan.close()
    with lma.Plan(opt, lma.lattice(w.scan[0], w.scan[1], Rx, Ry, f, w.offset_frac, w.L, window=win), det) as pp:
        pimg, t_plain = timed(lambda: pp.plain_image(v, device=True))
        pimg = pimg.cpu().numpy()
    log(f"paper-shaped: plain {t_plain:.2f} s for {win[2] * win[3]} probes")
    n_probes = w.scan[0] * w.scan[1]
    lma_rate = n_probes / t_lma
    plain_rate = win[2] * win[3] / t_plain
    err = {name: float(np.linalg.norm(lma_win[r] - pimg[r]) / np.linalg.norm(pimg[r]))
           for r, (name, _, _) in enumerate(w.detectors)}
    res = {
        "study": "paper-shaped stand-in: 1024^2 px over 84.536 x 79.941 A, scan 424x400, I=P+p/2, f=2, L=59, "
                 "200 kV, 26 mrad, Z=100 A, Cs=-2000 A, synthetic FCC specimen, 50 slices of 2 A, one configuration",
        "translates": info.n_rows, "probes": n_probes, "detector_pixels": info.n_pix,
        "basis_GB": info.n_rows * info.n_pix * 8 / 1e9, "probe_residual": info.max_residual,
        "contract_K": info.contract_k,
        "lma_seconds": t_lma, "lma_propagate_seconds": t_prop, "lma_contract_seconds": t_img,
        "lma_pixels_per_s": lma_rate,
        "plain_window": list(win), "plain_seconds": t_plain, "plain_pixels_per_s": plain_rate,
        "speedup_vs_plain": lma_rate / plain_rate,
        "lma_vs_plain_rel_l2_on_window": err}
    if emit:
        print(json.dumps(res), flush=True)
    return res


def _large_slices(args):
    """Slices [lo, hi) of the large workload's configuration-0 potential (the generator's own
    per-slice computation, run in a worker)."""
    from synth import WORKLOADS
    from synth.specimen import atom_sites, phonon_positions, potential_from_atoms
    lo, hi = args
    w = WORKLOADS["large"]
    sites, amps = atom_sites(w)
    return potential_from_atoms(w, phonon_positions(w, 0, sites), amps, range(lo, hi))


_LARGE_ORACLE = {}


def _large_oracle_wave(job):
    """An FP64 oracle exit spectrum at the large workload (a translate of psi_0 or a probe)."""
    import numpy as np
    from oracle.lma import translate_wave
    from oracle.multislice import multislice
    key, pos = job
    st, v = _LARGE_ORACLE["st"], _LARGE_ORACLE["v"]
    return key, np.fft.fft2(multislice(translate_wave(st, st.spec0, pos), v, st.sigma, st.prop))


def large_subscan(window=(120, 120, 16, 16), steps=1):
    """The large precision workload on a 16 x 16-probe sub-scan (2048^2 px over 204.8 A, 250
    slices, 300 kV, 25 mrad, defocus -50 A, translates every 4 px, L = 144, one phonon
    configuration): STEM pixels/s of the LMA image (propagation of the sub-scan's translates and
    the contraction) with the basis stored as split BF16 and as FP32, the slice passes' HBM
    roofline, and the error against the FP64 oracle of one LMA pixel formed from its 15 nearest
    translates (FP32 and split BF16) and one plain pixel."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from oracle import physics as ph
    from oracle.lma import Lattice, least_squares
    from oracle.multislice import Setup
    from synth import WORKLOADS

    w = WORKLOADS["large"]
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    step = -(-w.nslices // cores)
    log(f"large: potential ({w.nslices} x {w.nx}^2) on {cores} processes")
    with ProcessPoolExecutor(cores) as ex:
        v = np.concatenate(list(ex.map(_large_slices, [(lo, min(lo + step, w.nslices))
                                                       for lo in range(0, w.nslices, step)])))
    vd = torch.from_numpy(v).cuda()
    lam, sig = lma.electron_constants(w.kv)
    rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
    opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)
    R = (w.nx // w.basis_px, w.ny // w.basis_px)
    det = lma.detectors(rings)
    res = {"study": ("large workload, 16 x 16-probe sub-scan: 2048^2 px over 204.8 A, 250 slices of 2 A, FCC "
                     "{29,79} V*A random alloy, 300 kV, 25 mrad, defocus -50 A, translates every 4 px, L=144, one "
                     "phonon configuration"), "window": list(window)}
    for name, prec in (("split_bf16", lma.LMA_GEMM_SPLIT_BF16), ("fp32", lma.LMA_GEMM_FP32)):
        lat = lma.lattice(w.scan[0], w.scan[1], R[0], R[1], 1, w.offset_frac, w.L, prec, window=window)
        with lma.Plan(opt, lat, det) as plan:
            info = plan.info()
            img = torch.zeros(plan.image_shape(), dtype=torch.float64, device="cuda")
            plan.propagate(vd)                                   # first launches
            plan.probe_image(img)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.propagate(vd)
                plan.probe_image(img)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / steps
            plan.set_timing(True)
            plan.propagate(vd)
            plan.probe_image(img)
            kt = plan.timing(reset=True)
            plan.set_timing(False)
            n_probes = window[2] * window[3]
            row = {"seconds": t, "stem_pixels_per_s": n_probes / t, "translates": info.n_rows,
                   "detector_pixels": info.n_pix, "basis_GB": info.n_rows * info.n_pix * 8 / 1e9,
                   "probe_residual": info.max_residual, "batch": info.batch,
                   "kernels_ms": {k: {"launches": a, "total_ms": b} for k, (a, b) in kt.items()},
                   "contraction": contraction_roofline(plan, info, kt, split=prec == lma.LMA_GEMM_SPLIT_BF16)}
            XY = w.nx * w.ny
            batches = -(-info.n_rows // info.batch)
            wpl = info.n_rows / batches
            tw = info.tile_width
            kept = 1.0 - max(0, info.gap_hi // tw - (-(-info.gap_lo // tw))) * tw / w.nx
            first = 1.0 - max(0, info.input_gap_hi // tw - (-(-info.input_gap_lo // tw))) * tw / w.nx
            for pname in ("row_pass", "col_pass"):
                if pname not in kt:
                    continue
                n, ms = kt[pname]
                if pname == "row_pass":
                    rd = ((w.nslices - 1) * kept + first) / w.nslices
                    b = wpl * XY * 8 * (rd + kept) + XY * 8
                else:
                    b = (wpl * XY * 16 + XY * 8) * kept
                row[pname] = {"avg_launch_ms": ms / n, "algorithmic_bytes_per_launch": b,
                              "achieved_GBs": b / (ms / n * 1e-3) / 1e9,
                              "frac": b / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS}
            res[name] = row
            log(f"large: {name}: {t:.2f} s per image, {n_probes / t:.1f} STEM pixels/s")
    # one LMA pixel (L = 15) and one plain pixel against the FP64 oracle, 16 oracle waves
    probe = (window[0] + 3, window[1] + 5)
    L15 = 15
    px = {}
    for name, prec in (("fp32", lma.LMA_GEMM_FP32), ("split_bf16", lma.LMA_GEMM_SPLIT_BF16)):
        lat = lma.lattice(w.scan[0], w.scan[1], R[0], R[1], 1, w.offset_frac, L15, prec, window=(probe[0], probe[1], 1, 1))
        with lma.Plan(opt, lat, det) as plan:
            plan.propagate(vd)
            px[name] = plan.probe_image()[:, 0, 0]
            if name == "fp32":
                ppx = plan.plain_image(vd, device=True)[:, 0, 0].cpu().numpy()
    st = Setup(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs, w.scan,
               rings)
    ol = Lattice(st, R, 1, w.offset_frac, L15)
    nbr = ol.nearest(*probe)
    jobs = [((ta, tb), tuple(float(c) for c in ol.translate_position(ta, tb))) for ta, tb in nbr]
    jobs.append(("plain", st.probe_position(*probe)))
    _LARGE_ORACLE.update(st=st, v=v)
    log(f"large: FP64 oracle, {len(jobs)} waves on {min(cores, len(jobs))} processes")
    t0 = time.perf_counter()
    with ProcessPoolExecutor(min(cores, len(jobs))) as ex:
        waves = dict(ex.map(_large_oracle_wave, jobs))
    t_oracle = time.perf_counter() - t0
    _LARGE_ORACLE.clear()
    alpha = least_squares(st, ol, st.spec0, *probe)[0]
    ref = ph.detector_values(sum(c * waves[t] for c, t in zip(alpha, nbr)), st.masks)
    pref = ph.detector_values(waves["plain"], st.masks)
    res["error_vs_oracle"] = {
        "lma_pixel": list(probe), "L": L15,
        "lma_pixel_rel_err_fp32": [float(x) for x in np.abs(px["fp32"] - ref) / np.abs(ref)],
        "lma_pixel_rel_err_split_bf16": [float(x) for x in np.abs(px["split_bf16"] - ref) / np.abs(ref)],
        "plain_pixel_rel_err": [float(x) for x in np.abs(ppx - pref) / np.abs(pref)],
        "oracle_wall_s": t_oracle, "oracle_waves": len(jobs), "oracle_processes": min(cores, len(jobs))}
    return res


def uneven(n_specimens=64):
    """The uneven batch: n independent specimens of mixed grid sizes, slice counts and scans
    (synth.specimen.uneven_batch). Each forms the LMA image of a window of its scan: 16 x 16
    probes, or fewer when probes are sparser than translates (16 P / R per side, at least 2),
    so that every specimen propagates a few hundred translates. Timed with potentials
    resident in HBM, host planning excluded: (a) plan after plan, eager launches; (b) the
    same plans as one lma_batch graph launch; (c) plans built with LMA_AUTOTUNE | LMA_GRAPH,
    plan after plan from captured graphs; (d) those plans as one lma_batch launch; (e) the
    eager-layout plans as one grouped lma_batch (plans of one length class share each slice's
    row and column pass launch); (f) the autotuned plans grouped. Each image is checked
    against (a)."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth.specimen import potential_slices, uneven_batch

    ws = uneven_batch(n_specimens)
    log(f"uneven: generating {len(ws)} specimens")
    with ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        pots = [torch.from_numpy(v).cuda() for v in ex.map(potential_slices, ws)]
    sides = sorted({w.nx for w in ws})
    tuning = {}
    for n in sides:
        tuning[n] = lma.autotune(n, n)
        log(f"uneven: autotune {n}^2 -> {tuning[n]}")

    def window_of(w):
        R = w.nx // w.basis_px
        side = max(2, min(16, (16 * w.scan[0]) // R))
        return (0, 0, side, side)

    def build(flags):
        plans = []
        for w in ws:
            lam, sig = lma.electron_constants(w.kv)
            opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)
            (Rx, Ry), f = w.lattice_size()
            lat = lma.lattice(w.scan[0], w.scan[1], Rx, Ry, f, w.offset_frac, w.L, window=window_of(w))
            rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
            plans.append(lma.Plan(opt, lat, lma.detectors(rings), flags=flags))
        return plans

    def images(plans, imgs):
        for p, im in zip(plans, imgs):
            p.probe_image(im)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    nsl = [w.nslices for w in ws]
    log("uneven: building plans (eager layout)")
    plans = build(0)
    rows = sum(p.n_rows for p in plans)
    pixels = sum(int(np.prod(p.image_shape()[1:])) for p in plans)
    wave_slices = sum(p.n_rows * w.nslices for p, w in zip(plans, ws))
    imgs = [torch.zeros(p.image_shape(), dtype=torch.float64, device="cuda") for p in plans]

    def eager_round():
        for p, v in zip(plans, pots):
            p.propagate(v)
        images(plans, imgs)

    eager_round()                                   # first launches of every kernel shape
    t_eager = timed(eager_round)
    ref = [im.cpu().numpy() for im in imgs]
    batch = lma.Batch(plans, nsl)
    batch.propagate(pots)                           # capture
    images(plans, imgs)
    t_batch = timed(lambda: (batch.propagate(pots), images(plans, imgs)))
    err_batch = max(float(np.abs(im.cpu().numpy() - r).max() / np.abs(r).max()) for im, r in zip(imgs, ref))
    batch.close()
    log("uneven: grouped batch (eager layout)")
    batch = lma.Batch(plans, nsl, grouped=True)
    batch.propagate(pots)
    images(plans, imgs)
    t_grouped = timed(lambda: (batch.propagate(pots), images(plans, imgs)))
    err_grouped = max(float(np.abs(im.cpu().numpy() - r).max() / np.abs(r).max()) for im, r in zip(imgs, ref))
    batch.close()
    for p in plans:
        p.close()
    del plans
    log("uneven: building plans (autotuned layout, captured graphs)")
    plans = build(lma.LMA_AUTOTUNE | lma.LMA_GRAPH)
    for _ in range(2):                              # eager, then captured
        eager_round()
    t_graph = timed(eager_round)
    batch = lma.Batch(plans, nsl)
    batch.propagate(pots)
    images(plans, imgs)
    t_tuned_batch = timed(lambda: (batch.propagate(pots), images(plans, imgs)))
    err_tuned = max(float(np.abs(im.cpu().numpy() - r).max() / np.abs(r).max()) for im, r in zip(imgs, ref))
    batch.close()
    log("uneven: grouped batch (autotuned layout)")
    batch = lma.Batch(plans, nsl, grouped=True)
    batch.propagate(pots)
    images(plans, imgs)
    t_tuned_grouped = timed(lambda: (batch.propagate(pots), images(plans, imgs)))
    err_tuned_grouped = max(float(np.abs(im.cpu().numpy() - r).max() / np.abs(r).max()) for im, r in zip(imgs, ref))
    batch.close()
    for p in plans:
        p.close()
    res = {"eager": t_eager, "batch_graph": t_batch, "tuned_plan_graphs": t_graph, "tuned_batch_graph": t_tuned_batch,
           "grouped_batch": t_grouped, "tuned_grouped_batch": t_tuned_grouped}
    print(json.dumps({
        "study": f"uneven batch: {len(ws)} specimens, sides {sides} at 0.1 A/px, 20-200 slices of 2 A, FCC "
                 "{14,29,79} V*A, 200 kV, 20 mrad, translates every 4 px, L=144, scans 32-128 per side; "
                 "LMA image of a scan window per specimen",
        "specimens_by_side": {str(n): sum(1 for w in ws if w.nx == n) for n in sides},
        "translates": rows, "probes": pixels, "translate_slices": wave_slices,
        "autotune": {str(n): tuning[n] for n in sides},
        "seconds": res,
        "stem_pixels_per_s": {k: pixels / t for k, t in res.items()},
        "translate_slices_per_s": {k: wave_slices / t for k, t in res.items()},
        "max_rel_diff_vs_eager": {"batch_graph": err_batch, "tuned_batch_graph": err_tuned,
                                  "grouped_batch": err_grouped, "tuned_grouped_batch": err_tuned_grouped}}), flush=True)


def contraction_roofline(plan, info, kt, split=False):
    """Flop rate of the contraction launch against the MFMA peak of its data type. Useful
    (algorithmic) flops: 8 real flops per complex multiply-add, |P| L D of them; with the basis
    stored as split BF16 each real product is three bf16 products (hi hi, hi lo, lo hi), so its
    algorithmic count is 3 x that. `frac` is on those. Implemented flops (MFMA kernel): every
    4 x 4-probe sub-block multiplies a 16 x K coefficient block (K = contract_k translates, zero
    where a translate is not a neighbour) into 16-pixel slabs of each detector-pixel chunk: FP32,
    four real 16x16x4 products per K-step of 4 translates; split BF16, twelve bf16 16x16x16
    products per 16 translates; reported beside it."""
    name = "contract_mfma" if info.contract_kernel else "contract"
    if name not in kt:
        return None
    launches, total_ms = kt[name]
    avg_s = total_ms / launches * 1e-3
    _, mask = plan.detector_pixels()
    # chunks: runs of one ring mask in the sorted pixel list, cut every 256 pixels
    slabs = 0
    run = 1
    for i in range(1, len(mask) + 1):
        if i == len(mask) or mask[i] != mask[i - 1]:
            full, rest = divmod(run, 256)
            slabs += full * 16 + -(-rest // 16)
            run = 1
        else:
            run += 1
    alg = 8.0 * info.n_probes * info.L * info.n_pix
    nks = info.contract_k // 4
    bf16 = split and nks <= 80
    alg_mfma = alg * (3 if bf16 else 1)
    peak, dt = (BF16_MFMA_PEAK_TFLOPS, "bf16") if bf16 else (FP32_MFMA_PEAK_TFLOPS, "f32")
    out = {"kernel": name, "avg_launch_ms": avg_s * 1e3, "algorithmic_tflop": alg / 1e12,
           "useful_tflops": alg / avg_s / 1e12, "L": info.L, "K": info.contract_k,
           "traffic": load_traffic(name), "algorithmic_bytes": 8.0 * info.n_rows * info.n_pix,
           "bound": "mfma", "mfma_dtype": dt, "achieved": alg_mfma / avg_s / 1e12, "peak": peak,
           "unit": "TFLOP/s", "frac": alg_mfma / avg_s / 1e12 / peak,
           "what": ("useful flops: 8 |P| L D" + (" x 3 bf16 products per real product" if bf16 else "") +
                    " per launch over its hipEvent-timed duration")}
    if info.contract_kernel:
        ww, wh = plan.window[2], plan.window[3]
        sub_blocks = 4 * (-(-ww // 8)) * (-(-wh // 8))
        if bf16:
            impl = sub_blocks * slabs * (-(-nks // 4)) * 12 * (2 * 16 * 16 * 16)
        else:
            impl = sub_blocks * slabs * nks * 4 * (2 * 16 * 16 * 4)
        out.update({"implemented_tflop": impl / 1e12, "implemented_tflops": impl / avg_s / 1e12,
                    "implemented_frac": impl / avg_s / 1e12 / peak, "density": info.L / info.contract_k})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="arrival rate of the serving leg (requests/s)")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests of the serving leg per precision")
    ap.add_argument("--no-paper-shaped", action="store_true", help="skip the paper-shaped LMA-vs-plain leg")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the extra step that times every launch with hipEvents")
    ap.add_argument("--spacing-study", action="store_true",
                    help="LMA at translate spacings 4, 8, 16 px against plain multislice (one configuration)")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="print the HBM-traffic summary (JSON) of four rocprofv3 --pmc output directories")
    ap.add_argument("--serve-c5", choices=("fp32", "split_bf16"),
                    help="serving with requests drawn from the other workloads' sizes (one precision per run)")
    ap.add_argument("--serve-rates", type=str, default="1,2,5,10,20,50,100,200",
                    help="arrival rates of --serve-c5 (requests/s, comma separated)")
    ap.add_argument("--serve", action="store_true",
                    help="p50/p99 latency of the request loop under Poisson arrivals of image and local-edit requests")
    ap.add_argument("--paper-shaped", action="store_true",
                    help="LMA against plain multislice in the paper's regime (1024^2, 424x400 scan, f=2)")
    ap.add_argument("--window-study", action="store_true",
                    help="LMA with translates propagated on 64, 128, 256 px windows against plain multislice")
    ap.add_argument("--large-subscan", action="store_true",
                    help="the large precision workload on a 16 x 16-probe sub-scan (split BF16 and FP32), with its "
                         "error against the FP64 oracle")
    ap.add_argument("--uneven", action="store_true",
                    help="64 specimens of mixed sizes: eager, one batch graph, autotuned plans with graphs")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="RUN_DIR",
                    help="per-kernel means and utilisations from rocprofv3 --pmc runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy kernel (HBM counter calibration)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        # the copies run on torch's current stream, so its events time them
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(3):
            b.copy_(a)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / 3
        nbytes = a.numel() * 8
        print(json.dumps({"copy_bytes_each_way": nbytes, "copies": 4, "ms_per_copy": ms,
                          "read_plus_write_GBps": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2310_16829_amd as lma
    from synth import WORKLOADS, potential_slices

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WORKLOADS[WORKLOAD]
    if args.paper_shaped:
        paper_shaped()
        return
    if args.serve:
        serve()
        return
    if args.serve_c5:
        prec = lma.LMA_GEMM_SPLIT_BF16 if args.serve_c5 == "split_bf16" else lma.LMA_GEMM_FP32
        rates = tuple(float(x) for x in args.serve_rates.split(","))
        print(json.dumps(serve_c5(prec, rates, n_requests=args.serve_requests)), flush=True)
        return
    if args.uneven:
        uneven()
        return
    if args.large_subscan:
        print(json.dumps(large_subscan()), flush=True)
        return
    if args.spacing_study:
        spacing_study(w)
        return
    if args.window_study:
        window_study(w)
        return
    K, W = args.steps, args.warmup
    n_cfg = w.n_phonons
    log(f"bench: generating {min(n_cfg, K + W + 1)} phonon potentials")
    pots = [torch.from_numpy(potential_slices(w, c)).cuda() for c in range(min(n_cfg, K + W + 1))]
    torch.cuda.synchronize()

    lam, sig = lma.electron_constants(w.kv)
    rings = [(a * 1e-3, b * 1e-3) for _, a, b in w.detectors]
    opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)
    R = (w.nx // w.basis_px, w.ny // w.basis_px)
    lat = lma.lattice(w.scan[0], w.scan[1], R[0], R[1], 1, w.offset_frac, w.L, batch=args.batch)
    t0 = time.perf_counter()
    plan = lma.Plan(opt, lat, lma.detectors(rings))
    t_build = time.perf_counter() - t0
    info = plan.info()
    n_probes = info.n_probes
    log(f"bench: plan built in {t_build:.2f} s: {info.n_rows} translates, D={info.n_pix}, batch={info.batch}, "
        f"residual {info.max_residual:.2e}, {info.device_bytes / 2**30:.1f} GiB")
    stream = torch.cuda.current_stream()
    img = torch.zeros(plan.image_shape(), dtype=torch.float64, device="cuda")
    pimg = torch.zeros_like(img)

    def lma_step(c):
        plan.propagate(pots[c % len(pots)])
        plan.probe_image(img, flags=lma.LMA_ACCUMULATE, weight=1.0 / n_cfg)

    def plain_step(c):
        plan.plain_image(pots[c % len(pots)], pimg, flags=lma.LMA_ACCUMULATE, weight=1.0 / n_cfg)

    def timed(step, label):
        for c in range(W):
            step(c)
        torch.cuda.synchronize()
        img.zero_()
        pimg.zero_()
        lat_ms = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for c in range(K):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            step(W + c)
            e1.record(stream)
            e1.synchronize()
            lat_ms.append(e0.elapsed_time(e1))
            log(f"bench: {label} step {c + 1}/{K}: {lat_ms[-1]:.1f} ms")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        # one more step with a hipEvent pair around every launch, for per-kernel durations
        # (kept out of the timed region)
        if args.no_kernel_timing:
            return elapsed, lat_ms, {}
        plan.timing(reset=True)
        plan.set_timing(True)
        step(W + K)
        kt = plan.timing(reset=True)
        plan.set_timing(False)
        return elapsed, lat_ms, kt

    el, lat_ms, kt = timed(lma_step, "lma")
    value = n_probes * K / el
    plain = None
    if not args.no_plain:
        pel, plat_ms, pkt = timed(plain_step, "plain")
        plain = {"value": n_probes * K / pel, "ms_per_step": 1e3 * pel / K,
                 "p50_ms": float(np.percentile(plat_ms, 50)), "p99_ms": float(np.percentile(plat_ms, 99))}
    # roofline of the dominant kernel: a slice pass reads and writes every pixel of every wave
    # of its launch once (16 B per pixel per wave) and reads one 8 B/pixel table, except in the
    # band gap (kx columns that the band-limited propagator zeroes): column passes skip its tile
    # columns, row passes write none of it and read none of it after the first slice
    dom = max(("row_pass", "col_pass"), key=lambda k: kt.get(k, (0, 0.0))[1])
    launches, total_ms = kt.get(dom, (1, float("nan")))
    XY = w.nx * w.ny
    n_waves = info.n_rows
    batches = -(-n_waves // info.batch)
    waves_per_launch = n_waves / batches
    tw = info.tile_width
    gap_tiles = max(0, info.gap_hi // tw - (-(-info.gap_lo // tw)))
    kept = 1.0 - gap_tiles * tw / w.nx
    # the first row pass reads what the initial waves wrote: all but the input spectrum's gap
    first_read = 1.0 - max(0, info.input_gap_hi // tw - (-(-info.input_gap_lo // tw))) * tw / w.nx
    if dom == "row_pass":
        read = ((w.nslices - 1) * kept + first_read) / w.nslices
        bytes_per_launch = waves_per_launch * XY * 8 * (read + kept) + XY * 8
    else:
        bytes_per_launch = (waves_per_launch * XY * 16 + XY * 8) * kept
    avg_s = total_ms / launches * 1e-3
    achieved = bytes_per_launch / avg_s / 1e9
    # both slice passes together (every row and column pass of the step): their algorithmic
    # bytes over their summed launch time
    read_avg = ((w.nslices - 1) * kept + first_read) / w.nslices
    row_bytes = waves_per_launch * XY * 8 * (read_avg + kept) + XY * 8
    col_bytes = (waves_per_launch * XY * 16 + XY * 8) * kept
    n_row, t_row = kt.get("row_pass", (0, 0.0))
    n_col, t_col = kt.get("col_pass", (0, 0.0))
    both_bytes = n_row * row_bytes + n_col * col_bytes
    both_s = (t_row + t_col) * 1e-3
    slice_passes = {"bound": "hbm", "kernels": ["row_pass", "col_pass"], "launches": [n_row, n_col],
                    "achieved": both_bytes / both_s / 1e9 if both_s > 0 else None, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": both_bytes / both_s / 1e9 / HBM_PEAK_GBS if both_s > 0 else None,
                    "algorithmic_bytes": both_bytes, "total_ms": t_row + t_col}
    traffic = load_traffic(dom)
    contraction = contraction_roofline(plan, info, kt)
    # the precision mode: the same configuration with the basis stored as split BF16 and the
    # contraction on the bf16 MFMA (propagation untimed), its launch time and its image error
    # against the FP32 basis
    split = None
    images = {}
    ref = torch.zeros_like(img)
    plan.propagate(pots[0])
    plan.probe_image(ref)
    images["fp32"] = ref.cpu().numpy()
    if not args.no_kernel_timing:
        slat = lma.lattice(w.scan[0], w.scan[1], R[0], R[1], 1, w.offset_frac, w.L, lma.LMA_GEMM_SPLIT_BF16,
                           batch=args.batch)
        with lma.Plan(opt, slat, lma.detectors(rings)) as sp:
            simg = torch.zeros_like(img)
            sp.propagate(pots[0])
            sp.probe_image(simg)
            sp.set_timing(True)
            for _ in range(3):
                sp.probe_image(simg)
            skt = sp.timing(reset=True)
            split = contraction_roofline(sp, sp.info(), skt, split=True)
        r, s_ = images["fp32"], simg.cpu().numpy()
        images["split_bf16"] = s_
        split["image_rel_l2_vs_fp32_basis"] = [float(np.linalg.norm(s_[i] - r[i]) / np.linalg.norm(r[i]))
                                               for i in range(r.shape[0])]
    out = {
        "metric": "STEM pixels/s, LMA vs plain multislice, same GPU at <=1e-4 rel err; p99 latency",
        "value": value,
        "unit": "STEM pixels/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("medium: 512x512 px over 51.2 A, 100 slices of 2 A, FCC a=4.05 A, amplitudes "
                                "{14,29,79} V*A, 200 kV, 20 mrad, scan 128x128, LMA translate spacing 4 px "
                                "(offset 1/2), L=144, 8 frozen-phonon configurations; one step = one configuration"),
                   "scan": [w.scan[0], w.scan[1]], "grid": [w.nx, w.ny], "slices": w.nslices,
                   "translates": n_waves, "L": w.L, "batch": info.batch},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "what": "one phonon configuration of the full image (propagate + probe_image)"},
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "lma_probe_residual": info.max_residual,
        "kernels_ms": {k: {"launches": v[0], "total_ms": v[1]} for k, v in kt.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "band_gap_columns": [info.gap_lo, info.gap_hi], "kept_fraction": kept,
                     "input_gap_columns": [info.input_gap_lo, info.input_gap_hi],
                     "avg_launch_ms": avg_s * 1e3},
        "slice_passes": slice_passes,
        "contraction": contraction,
        "contraction_split_bf16": split,
        "plan_build_s": t_build,
    }
    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline")
        torch.cuda.synchronize()
        out["cpu_baseline"] = cpu_baseline(w, n_waves, n_probes, plan, images)
        out["error_vs_oracle"] = out["cpu_baseline"].pop("error_vs_oracle")
        if split is not None:
            split["lma_pixel_rel_err_vs_oracle"] = out["error_vs_oracle"]["lma_pixel_rel_err_per_detector"]["split_bf16"]
    plan.close()
    del pots
    torch.cuda.empty_cache()
    if not args.no_serving:
        # loaded latency: the request loop under Poisson arrivals of mixed-size image and edit requests
        log("bench: serving leg")
        out["serving"] = serve(rates=(args.serve_rate,), n_requests=args.serve_requests, slots=4, emit=False,
                               cap_seconds=None)
    if not args.no_paper_shaped:
        log("bench: paper-shaped leg")
        out["paper_shaped"] = paper_shaped(emit=False)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

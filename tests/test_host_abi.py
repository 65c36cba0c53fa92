"""CPU tests of the C-ABI library: symbols, argument checks and the host planner (on host-only
plans) against the FP64 oracle. No device work is requested here."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2310_16829_amd as lma
from paper_2310_16829_amd import _lib
from oracle import physics as ph
from oracle.lma import LMA, Lattice, least_squares, translate_wave
from oracle.multislice import Setup
from synth import WORKLOADS
from tests._cases import det_rad, longest_zero_run, oracle_lattice, oracle_setup, rel_l2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "lma.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lma_status|void|const char\*)\s+(lma_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2310_16829_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, flags=re.M), f
                assert "oracle/" not in txt, f


def _plan_args(w, L=None, scan=None, R=None, f=1, offset=None, window=(0, 0, 0, 0), precision=0, nx=None, ny=None,
               lx=None, ly=None, batch=0, basis_kind=0, basis_param=0.0):
    lam, sig = lma.electron_constants(w.kv)
    opt = lma.optics(nx or w.nx, ny or w.ny, lx or w.lx, ly or w.ly, lam, sig, w.dz, w.bandlimit,
                     w.alpha_mrad * 1e-3, w.defocus, w.cs)
    scan = scan or w.scan
    if R is None:
        R = ((nx or w.nx) // w.basis_px * f, (ny or w.ny) // w.basis_px * f)
    lat = lma.lattice(scan[0], scan[1], R[0], R[1], f, offset or w.offset_frac, w.L if L is None else L, precision,
                      window, batch, basis_kind=basis_kind, basis_param=basis_param)
    det = lma.detectors(det_rad(w))
    return opt, lat, det


def test_electron_constants_match_oracle():
    for kv in (80.0, 200.0, 300.0):
        lam, sig = lma.electron_constants(kv)
        assert abs(lam - ph.electron_wavelength(kv)) < 1e-15
        assert abs(sig - ph.interaction_constant(kv)) < 1e-15
    with pytest.raises(lma.LmaError):
        lma.electron_constants(-1.0)


@pytest.mark.parametrize("case", ["tiny", "case2", "nonsquare", "f2_paper_style", "gaussian", "gaussian_sigma",
                                  "grid_96_by_640", "trigpoly_exact", "trigpoly_nearest", "trigpoly_offset"])
def test_host_plan_matches_oracle(case):
    w = WORKLOADS["tiny"]
    kw = {}
    okw = {}
    if case == "gaussian":       # u = g_sigma with the paper's sigma = lambda / (2 alpha_max)
        kw = dict(L=100, basis_kind=lma.LMA_BASIS_GAUSSIAN)
    elif case == "gaussian_sigma":   # an explicit sigma, Case 2 lattice
        kw = dict(scan=(16, 16), R=(8, 8), L=16, basis_kind=lma.LMA_BASIS_GAUSSIAN, basis_param=0.9)
    elif case == "grid_96_by_640":   # mixed-radix sides
        kw = dict(nx=96, ny=640, lx=9.6, ly=64.0, scan=(12, 80), R=(24, 160), L=16)
    elif case == "case2":        # P = 2 R_f: four coefficient sets
        kw = dict(scan=(16, 16), R=(8, 8), L=16)
    elif case == "nonsquare":    # nx != ny, lx != ly, Case 1 with c = 2 along x and 1 along y
        kw = dict(nx=128, ny=64, lx=12.8, ly=7.2, scan=(16, 16), R=(32, 16), L=24)
    elif case == "f2_paper_style":  # I = P + p/2, f = 2 (Sec. 4.2.3)
        kw = dict(scan=(32, 32), R=(32, 32), f=2, L=25, offset=(0.5, 0.5))
    elif case == "trigpoly_exact":   # phi_10 x phi_10 over all 21 x 21 translates: exact (Sec. 2)
        kw = dict(scan=(42, 42), R=(21, 21), L=441, offset=(0.0, 0.0), basis_kind=lma.LMA_BASIS_TRIGPOLY)
    elif case == "trigpoly_nearest":  # closed-form coefficients kept at the 81 nearest translates
        kw = dict(scan=(42, 42), R=(21, 21), L=81, offset=(0.0, 0.0), basis_kind=lma.LMA_BASIS_TRIGPOLY)
    elif case == "trigpoly_offset":   # non-square cell, degrees 10 and 6, offset lattice, f = 2
        kw = dict(nx=128, ny=64, lx=12.8, ly=7.2, scan=(21, 13), R=(42, 26), f=2, L=150, offset=(0.5, 0.5),
                  basis_kind=lma.LMA_BASIS_TRIGPOLY)
    opt, lat, det = _plan_args(w, **kw)
    plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    info = plan.info()
    st = Setup(opt.nx, opt.ny, opt.lx, opt.ly, opt.wavelength, opt.sigma, opt.dz, opt.bandlimit, opt.alpha_max,
               opt.defocus, opt.cs, (lat.px, lat.py), det_rad(w))
    ol = Lattice(st, (lat.rx, lat.ry), lat.f, (lat.offset_x, lat.offset_y), lat.L)
    assert (info.ncls_x, info.ncls_y) == (ol.ncls_x, ol.ncls_y)
    assert info.n_translates == ol.n_translates
    # probe spectrum, and the input wave's
    assert np.abs(plan.probe_spectrum() - st.spec0).max() < 1e-12
    trig = kw.get("basis_kind") == lma.LMA_BASIS_TRIGPOLY
    if trig:
        spec_u = ph.trigpoly_spectrum(st.nx, st.ny, st.lx, st.ly, (ol.Rfx - 1) // 2, (ol.Rfy - 1) // 2)
    elif kw.get("basis_kind"):
        sg = kw.get("basis_param") or st.wavelength / (2 * st.alpha_max)
        spec_u = ph.gaussian_spectrum(st.nx, st.ny, st.lx, st.ly, sg)
    else:
        spec_u = st.spec0
    assert np.abs(plan.input_wave_spectrum() - spec_u).max() < 1e-10 * np.abs(spec_u).max()
    # detector pixels and ring masks: bit-exact
    flat, mask = plan.detector_pixels()
    om = np.zeros(opt.nx * opt.ny, np.uint32)
    for r, m in enumerate(st.masks):
        om |= m.ravel().astype(np.uint32) << np.uint32(r)
    assert np.array_equal(np.sort(flat), np.nonzero(om)[0])
    assert np.array_equal(om[flat], mask)
    # translate positions
    pos = plan.translates()
    for t in (0, 1, ol.Rfx, ol.n_translates - 1):
        ta, tb = t % ol.Rfx, t // ol.Rfx
        ex = ol.translate_position(ta, tb)
        assert abs(pos[t, 0] - float(ex[0])) < 1e-12 and abs(pos[t, 1] - float(ex[1])) < 1e-12
    # neighbour lists (ordered, exact) and approximants of every coefficient set
    tr, al = plan.coefficients()
    lm = LMA(st, ol, spec_u=spec_u, coefficients="trigpoly" if trig else "least_squares")
    for sy in range(ol.ncls_y):
        for sx in range(ol.ncls_x):
            s = sy * ol.ncls_x + sx
            want = [tb * ol.Rfx + ta for ta, tb in ol.nearest(sx, sy)]
            assert list(tr[s]) == want
            appr = sum(a * translate_wave(st, spec_u, ol.translate_position(t % ol.Rfx, t // ol.Rfx))
                       for a, t in zip(al[s], tr[s]))
            assert rel_l2(appr, lm.approximant(sx, sy)) < 1e-8
    if case == "trigpoly_exact":
        assert info.max_residual < 1e-12 and max(lm.residual.values()) < 1e-12
    else:
        assert info.max_residual == pytest.approx(max(lm.residual.values()), rel=1e-6)


@pytest.mark.parametrize("case", ["tiny", "case2", "f2_paper_style", "nonsquare", "defocus_cs"])
def test_host_coefficients_equal_the_oracles(case):
    # where a translate set has full column rank its least-squares coefficients are unique (the
    # oracle's are pinned by the normal equations), so the planner's own QR / SVD solve must
    # return those coefficients, not only an equally good approximant (Sec. 4.2.2)
    w = WORKLOADS["tiny"]
    kw = {"tiny": {}, "case2": dict(scan=(16, 16), R=(8, 8), L=16),
          "f2_paper_style": dict(scan=(32, 32), R=(32, 32), f=2, L=25, offset=(0.5, 0.5)),
          "nonsquare": dict(nx=128, ny=64, lx=12.8, ly=7.2, scan=(16, 16), R=(32, 16), L=24),
          "defocus_cs": dict(scan=(16, 16), R=(16, 16), L=20)}[case]
    opt, lat, det = _plan_args(w, **kw)
    if case == "defocus_cs":            # a complex probe: defocus and spherical aberration
        opt = lma.optics(opt.nx, opt.ny, opt.lx, opt.ly, opt.wavelength, opt.sigma, opt.dz, opt.bandlimit,
                         opt.alpha_max, -60.0, 2.0e4)
    plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    st = Setup(opt.nx, opt.ny, opt.lx, opt.ly, opt.wavelength, opt.sigma, opt.dz, opt.bandlimit, opt.alpha_max,
               opt.defocus, opt.cs, (lat.px, lat.py), det_rad(w))
    ol = Lattice(st, (lat.rx, lat.ry), lat.f, (lat.offset_x, lat.offset_y), lat.L)
    tr, al = plan.coefficients()
    for sy in range(ol.ncls_y):
        for sx in range(ol.ncls_x):
            s = sy * ol.ncls_x + sx
            a_o, nbr, res = least_squares(st, ol, st.spec0, sx, sy)
            assert list(tr[s]) == [tb * ol.Rfx + ta for ta, tb in nbr]
            B = np.stack([translate_wave(st, st.spec0, ol.translate_position(ta, tb)).ravel() for ta, tb in nbr],
                         axis=1)
            sv = np.linalg.svd(B, compute_uv=False)
            assert sv[-1] > 1e-6 * sv[0]
            assert np.abs(np.asarray(al[s]) - a_o).max() <= 1e-9 * np.abs(a_o).max()


@pytest.mark.parametrize("case", ["medium", "tiny", "f2_paper_style"])
def test_mfma_layout_k_steps_cover_the_sub_block_union(case):
    # the banded-GEMM layout of the contraction (eqs. lma_approximation_exit1/2): a 4 x 4-probe
    # sub-block's K-steps are runs of 4 translates along x on each row of the union of its
    # probes' neighbour sets, so K = 4 x sum over rows of ceil(row span / 4). Counted here from
    # the oracle's neighbour sets of a sub-block away from the cell's edge (the layout is the
    # same for every sub-block).
    w = WORKLOADS["medium" if case == "medium" else "tiny"]
    kw = dict(scan=(32, 32), R=(32, 32), f=2, L=25, offset=(0.5, 0.5)) if case == "f2_paper_style" else {}
    opt, lat, det = _plan_args(w, **kw)
    info = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY).info()
    assert info.contract_kernel == 1
    st = Setup(opt.nx, opt.ny, opt.lx, opt.ly, opt.wavelength, opt.sigma, opt.dz, opt.bandlimit, opt.alpha_max,
               opt.defocus, opt.cs, (lat.px, lat.py), det_rad(w))
    ol = Lattice(st, (lat.rx, lat.ry), lat.f, (lat.offset_x, lat.offset_y), lat.L)
    a0, b0 = lat.px // 8 * 4, lat.py // 8 * 4
    span = {}
    for b in range(b0, b0 + 4):
        for a in range(a0, a0 + 4):
            for ta, tb in ol.nearest(a, b):
                lo, hi = span.get(tb, (ta, ta))
                span[tb] = (min(lo, ta), max(hi, ta))
    assert all(hi - lo < ol.Rfx // 2 for lo, hi in span.values())     # no wrap-around here
    nks = sum(-(-(hi - lo + 1) // 4) for lo, hi in span.values())
    assert info.contract_k == 4 * nks
    if case == "medium":
        assert info.contract_k == 272 and lat.L == 144   # the density L / K = 0.53 the bench line reports


def test_window_rows_are_the_union_of_neighbour_sets():
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w, window=(3, 14, 4, 2), L=16)
    plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    st = oracle_setup(w)
    ol = oracle_lattice(w, st, L=16)
    need = set()
    for b in range(14, 16):
        for a in range(3, 7):
            need.update(tb * ol.Rfx + ta for ta, tb in ol.nearest(a, b))
    assert sorted(need) == list(plan.rows())
    assert plan.image_shape() == (4, 2, 4)


@pytest.mark.parametrize("bad", [
    dict(nx=80), dict(nx=100), dict(nx=4096), dict(scan=(12, 16)), dict(L=0), dict(L=5000), dict(offset=(0.3, 0.5)),
    dict(window=(10, 0, 8, 4)), dict(f=3, R=(32, 32)), dict(batch=-1),
])
def test_invalid_arguments_are_rejected(bad):
    w = WORKLOADS["tiny"]
    kw = dict(bad)
    nx = kw.pop("nx", None)
    batch = kw.pop("batch", 0)
    opt, lat, det = _plan_args(w, nx=nx, batch=max(batch, 0), **kw)
    if batch < 0:
        lat.batch = batch
    with pytest.raises(lma.LmaError) as e:
        lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    assert e.value.status in (_lib.LMA_ERR_ARG, _lib.LMA_ERR_UNSUPPORTED)


def test_invalid_detectors_and_optics_are_rejected():
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    for rings in ([(0.02, 0.01)], [], [(0, 0.1)] * 9, [(-0.01, 0.02)]):
        with pytest.raises(lma.LmaError):
            lma.Plan(opt, lat, lma.detectors(rings), flags=lma.LMA_HOST_ONLY)
    for field, val in (("wavelength", 0.0), ("dz", -2.0), ("bandlimit", 1.5), ("alpha_max", 0.0), ("lx", float("nan"))):
        o2 = lma.optics(opt.nx, opt.ny, opt.lx, opt.ly, opt.wavelength, opt.sigma, opt.dz, opt.bandlimit,
                        opt.alpha_max)
        setattr(o2, field, val)
        with pytest.raises(lma.LmaError):
            lma.Plan(o2, lat, det, flags=lma.LMA_HOST_ONLY)


def test_host_only_plan_refuses_device_work():
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    v = np.zeros((2, w.ny, w.nx), np.float32)
    for call in (lambda: plan.propagate(v), lambda: plan.probe_image(), lambda: plan.plain_image(v),
                 lambda: plan.basis_rows(0, 1), lambda: plan.save_basis(os.devnull),
                 lambda: plan.load_basis(os.devnull)):
        with pytest.raises(lma.LmaError) as e:
            call()
        assert e.value.status == _lib.LMA_ERR_STATE


@pytest.mark.parametrize("side,bandlimit", [(128, None), (96, None), (640, None), (128, 1.0), (128, 0.3)])
def test_kx_gaps_match_the_oracle(side, bandlimit):
    # the band gap (columns where the band-limited propagator vanishes for every ky and no ring
    # has a pixel) and the input gap (columns where the probe spectrum vanishes), against the
    # oracle's propagator, ring masks and probe spectrum
    w = WORKLOADS["tiny"]
    bl = bandlimit or w.bandlimit
    lx = w.lx * side / w.nx
    lam, sig = lma.electron_constants(w.kv)
    rings = det_rad(w)
    opt = lma.optics(side, side, lx, lx, lam, sig, w.dz, bl, w.alpha_mrad * 1e-3, w.defocus, w.cs)
    lat = lma.lattice(16, 16, 16, 16, 1, w.offset_frac, 9)
    i = lma.Plan(opt, lat, lma.detectors(rings), flags=lma.LMA_HOST_ONLY).info()
    st = Setup(side, side, lx, lx, lam, sig, w.dz, bl, w.alpha_mrad * 1e-3, w.defocus, w.cs, (16, 16), rings)
    band = np.all(st.prop == 0, axis=0) & ~np.any([m.any(axis=0) for m in st.masks], axis=0)
    assert (i.gap_lo, i.gap_hi) == longest_zero_run(band)
    assert (i.input_gap_lo, i.input_gap_hi) == longest_zero_run(np.all(st.spec0 == 0, axis=0))
    # the aperture (20 mrad) lies inside the band: the input gap holds the band gap
    assert i.input_gap_lo <= i.gap_lo and i.gap_hi <= i.input_gap_hi


def test_footprint_grows_with_slices_and_basis():
    w = WORKLOADS["medium"]
    opt, lat, det = _plan_args(w)
    b1 = lma.footprint(opt, lat, det, 1)
    b100 = lma.footprint(opt, lat, det, 100)
    assert b100 > b1 > 16384 * 90081 * 8          # the resident basis alone is ~11.8 GB
    with pytest.raises(lma.LmaError):
        lma.footprint(opt, lat, det, 0)


# ---------------------------------------------------------------------------------------
# rectangle partition under a residency budget (Sec. 4.2.4)
# ---------------------------------------------------------------------------------------
def _partition_case(w, M, **kw):
    from oracle.partition import multislice_calls, rectangles, union
    opt, lat, det = _plan_args(w, **kw)
    with lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY) as p:
        info = p.info()
        assert info.partitioned == 0 and info.multislice_calls == info.n_rows
        D, window, stencil = info.n_pix, p.window, info.contract_kernel
    lat.hbm_budget_bytes = M * D * 8
    with lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY) as p:
        info = p.info()
    st = oracle_setup(w, **{k: v for k, v in kw.items() if k in ("nx", "ny", "lx", "ly", "scan")})
    ol = oracle_lattice(w, st, **{k: v for k, v in kw.items() if k in ("R", "f", "offset", "L")})
    a0, b0, ww, wh = window
    sets = {(a, b): ol.nearest((a0 + a) % st.Px, (b0 + b) % st.Py) for b in range(wh) for a in range(ww)}
    parts = rectangles(sets, (0, 0, ww, wh), M)
    assert info.partitioned == 1
    assert (info.part_w, info.part_h) == (max(a for a, _ in parts[0]) + 1, max(b for _, b in parts[0]) + 1)
    # the same parts in the same order
    assert info.n_parts == len(parts)
    pw, ph = info.part_w, info.part_h
    for j, q in enumerate(parts):
        a_lo, b_lo = min(a for a, _ in q), min(b for _, b in q)
        assert (a_lo, b_lo) == ((j % -(-ww // pw)) * pw, (j // -(-ww // pw)) * ph)
    assert info.n_parts == len(parts)
    assert info.multislice_calls == multislice_calls(sets, parts)
    assert info.resident_rows == max(len(union(sets, q)) for q in parts) <= M
    return info, parts


def test_partition_case1_matches_oracle_rectangles():
    # tiny workload (Case 1, two translates per probe step), MFMA contraction; rectangles of
    # any side (probes outside a rectangle in its super-tiles are not formed)
    info, parts = _partition_case(WORKLOADS["tiny"], 600)
    assert info.contract_kernel == 1 and info.n_parts > 1
    for M in (150, 260, 400):
        _partition_case(WORKLOADS["tiny"], M)


def test_partition_case2_three_sets_matches_oracle_rectangles():
    # Case 2 with three coefficient sets per axis: per-pixel contraction
    w = WORKLOADS["tiny"]
    info, parts = _partition_case(w, 30, scan=(48, 48), R=(16, 16), L=12, window=(5, 7, 13, 10))
    assert info.contract_kernel == 0 and info.n_parts > 1


def test_partition_budget_below_one_rectangle_is_refused():
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    lat.hbm_budget_bytes = 100 * 8   # far less than one row of D pixels
    with pytest.raises(lma.LmaError) as e:
        lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    assert e.value.status == _lib.LMA_ERR_OOM


# ---------------------------------------------------------------------------------------
# serving loop: argument checks and host-side bookkeeping (no device work)
# ---------------------------------------------------------------------------------------
def test_server_arguments():
    with pytest.raises(lma.LmaError) as e:
        lma.Server(0, 4, 1 << 30)
    assert e.value.status == _lib.LMA_ERR_ARG
    with pytest.raises(lma.LmaError):
        lma.Server(2, 0, 1 << 30)
    with pytest.raises(lma.LmaError):
        lma.Server(2, 4, 0)
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    need = lma.footprint(opt, lat, det, w.nslices)
    with lma.Server(2, 4, need - 1) as s:
        with pytest.raises(lma.LmaError) as e:
            s.build(0, opt, lat, det, w.nslices)          # can never be admitted
        assert e.value.status == _lib.LMA_ERR_OOM
        with pytest.raises(lma.LmaError) as e:
            s.build(4, opt, lat, det, w.nslices)          # no such specimen slot
        assert e.value.status == _lib.LMA_ERR_ARG
        with pytest.raises(lma.LmaError) as e:
            s.wait(99)
        assert e.value.status == _lib.LMA_ERR_ARG
        assert s.in_use() == 0


def test_server_reports_request_failures():
    # a request on a specimen that was never built fails with LMA_ERR_STATE; the server keeps
    # running and a release of an empty slot succeeds
    w = WORKLOADS["tiny"]
    with lma.Server(2, 4, 1 << 30) as s:
        v = np.zeros((w.nslices, w.ny, w.nx), dtype=np.float32)
        img = np.zeros((4, 16, 16))
        t = s.image(1, v, img)
        with pytest.raises(lma.LmaError) as e:
            s.wait(t)
        assert e.value.status == _lib.LMA_ERR_STATE and "not resident" in str(e.value)
        lat, svc = s.wait(s.release(1))
        assert lat >= svc >= 0.0
        assert s.in_use() == 0


def test_server_refuses_a_second_build_of_a_resident_specimen():
    # host-only specimens: a BUILD of a specimen that is already resident fails with
    # LMA_ERR_STATE and neither replaces its plan nor admits more bytes; after a RELEASE the
    # same slot builds again
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    need = lma.footprint(opt, lat, det, w.nslices)
    with lma.Server(2, 2, 3 * need) as s:
        s.wait(s.build(0, opt, lat, det, w.nslices, flags=lma.LMA_HOST_ONLY))
        assert s.in_use() == need
        n_rows = s.plan_info(0).n_rows
        with pytest.raises(lma.LmaError) as e:
            s.wait(s.build(0, opt, lat, det, w.nslices, flags=lma.LMA_HOST_ONLY))
        assert e.value.status == _lib.LMA_ERR_STATE and "already resident" in str(e.value)
        assert s.in_use() == need and s.plan_info(0).n_rows == n_rows
        s.wait(s.release(0))
        assert s.in_use() == 0
        s.wait(s.build(0, opt, lat, det, w.nslices, flags=lma.LMA_HOST_ONLY))
        assert s.in_use() == need
        # a host-only specimen answers image requests with LMA_ERR_STATE
        with pytest.raises(lma.LmaError) as e:
            s.wait(s.image(0, np.zeros((w.nslices, w.ny, w.nx), np.float32), np.zeros((4, 16, 16))))
        assert e.value.status == _lib.LMA_ERR_STATE


def test_server_wait_twice_returns_an_error():
    # each ticket is waited for once; a second wait returns LMA_ERR_ARG at once instead of
    # blocking, and so does a ticket that was never issued
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    with lma.Server(1, 2, 1 << 40) as s:
        t = s.build(1, opt, lat, det, w.nslices, flags=lma.LMA_HOST_ONLY)
        s.wait(t)
        with pytest.raises(lma.LmaError) as e:
            s.wait(t)
        assert e.value.status == _lib.LMA_ERR_ARG and "already waited" in str(e.value)
        with pytest.raises(lma.LmaError) as e:
            s.wait(t + 1000)
        assert e.value.status == _lib.LMA_ERR_ARG


def test_server_build_failure_returns_its_bytes():
    # on a machine without a GPU the build itself fails; its admitted footprint is returned
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present: the build would succeed")
    except ImportError:
        pass
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    with lma.Server(1, 2, 1 << 34) as s:
        with pytest.raises(lma.LmaError) as e:
            s.wait(s.build(0, opt, lat, det, w.nslices))
        assert e.value.status == _lib.LMA_ERR_DEVICE
        assert s.in_use() == 0


def test_window_tables_match_the_oracle():
    # option (ii): the window spectrum is the DFT of u cropped to a window centred on a
    # translate; the window propagator keeps the cell's band limit
    from oracle.lma import LMA as OLMA
    w = WORKLOADS["tiny"]
    for win in ((64, 32), (128, 128), (96, 16)):
        opt, lat, det = _plan_args(w)
        lat.prop_nx, lat.prop_ny = win
        plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
        i = plan.info()
        assert (i.prop_nx, i.prop_ny) == win
        st = oracle_setup(w)
        ol = oracle_lattice(w, st)
        om = OLMA(st, ol, window=win)
        t = (5, 2)
        cx, cy = om.window_origin(*t)
        u = translate_wave(st, st.spec0, ol.translate_position(*t))
        ref = np.fft.fft2(u[np.ix_((cy + np.arange(win[1])) % 128, (cx + np.arange(win[0])) % 128)])
        got = plan.window_spectrum()
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # every window has the same wave only when translates sit on pixels: 48 translates over
    # 128 pixels do not
    opt, lat, det = _plan_args(w, R=(48, 48), offset=(0.0, 0.0))
    lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    lat.prop_nx, lat.prop_ny = 64, 64
    with pytest.raises(lma.LmaError, match="translates on pixels"):
        lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    for bad in ((100, 64), (256, 64), (64, 0)):
        opt, lat, det = _plan_args(w)
        lat.prop_nx, lat.prop_ny = bad
        with pytest.raises(lma.LmaError):
            lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)


def test_autotune_and_batch_argument_checks():
    # checked before any device work, so these run without a GPU
    with pytest.raises(lma.LmaError) as e:
        lma.autotune(100, 100)
    assert e.value.status == _lib.LMA_ERR_UNSUPPORTED
    t = _lib.lma_tuning()
    assert lma.lib().lma_autotune(128, 128, -1, None, ctypes.byref(t)) != 0
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    out = ctypes.c_void_p()
    one = (ctypes.c_int32 * 1)(10)
    assert lma.lib().lma_batch_create(None, 1, one, None, ctypes.byref(out)) == _lib.LMA_ERR_ARG
    hs = (ctypes.c_void_p * 1)(plan._h.value)
    assert lma.lib().lma_batch_create(hs, 0, one, None, ctypes.byref(out)) == _lib.LMA_ERR_ARG
    # a host-only plan has no device state (or, without a GPU, there is no device at all)
    assert lma.lib().lma_batch_create(hs, 1, one, None, ctypes.byref(out)) in (_lib.LMA_ERR_STATE, _lib.LMA_ERR_DEVICE)
    assert not out.value


def test_3d_4d_outputs_refuse_host_only_plans():
    w = WORKLOADS["tiny"]
    opt, lat, det = _plan_args(w)
    plan = lma.Plan(opt, lat, det, flags=lma.LMA_HOST_ONLY)
    with pytest.raises(lma.LmaError):
        plan.probe_patterns()
    with pytest.raises(lma.LmaError):
        plan.probe_radial(0.005, 10)
    img = np.zeros((10, 16, 16))
    assert lma.lib().lma_probe_radial(plan._h, 0.0, 10, ctypes.c_void_p(img.ctypes.data), 0, 1.0) != 0

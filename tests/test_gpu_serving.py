"""GPU tests of the serving loop (lma_server): every result is the same alone and in the mix,
and new specimens are admitted by device footprint."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import paper_2310_16829_amd as lma
from synth import WORKLOADS, potential_slices
from tests._cases import det_rad, oracle_lattice, oracle_setup
from tests.test_gpu_parity import PAPER_RINGS, TOL32, image_errors

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", [0, 1])
def test_basis_save_and_load(tmp_path, precision):
    # a propagated basis written to a file and read by a fresh plan of the same layout gives the
    # same rows bit for bit and the same images; a plan of another layout (detectors, encoding), a
    # truncated file and a file of another kind are refused before anything reaches the device
    from paper_2310_16829_amd import _lib
    prec = (lma.LMA_GEMM_FP32, lma.LMA_GEMM_SPLIT_BF16)[precision]
    w = WORKLOADS["tiny"]
    lam, sig = lma.electron_constants(w.kv)
    opt = lma.optics(w.nx, w.ny, w.lx, w.ly, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3)
    det = lma.detectors(det_rad(w))
    lat = lma.lattice(16, 16, 32, 32, 1, (0.5, 0.5), 36, prec)
    v = potential_slices(w, 0)
    say(f"basis file, precision {prec}")
    a = lma.Plan(opt, lat, det)
    a.propagate(v)
    img, rows = a.probe_image(), a.basis_rows(0, a.n_rows)
    path = str(tmp_path / "tiny.basis")
    a.save_basis(path)
    a.close()
    b = lma.Plan(opt, lat, det)
    with pytest.raises(lma.LmaError):
        b.probe_image()                                   # nothing propagated or loaded yet
    b.load_basis(path)
    assert np.array_equal(b.basis_rows(0, b.n_rows), rows)
    assert np.allclose(b.probe_image(), img, rtol=1e-12, atol=0)   # FP64 atomics: sum order varies
    b.close()
    data = open(path, "rb").read()
    cut, junk = str(tmp_path / "cut.basis"), str(tmp_path / "junk.basis")
    open(cut, "wb").write(data[:-8])
    open(junk, "wb").write(b"not a basis" * 16)
    other_prec = lma.lattice(16, 16, 32, 32, 1, (0.5, 0.5), 36,
                             lma.LMA_GEMM_FP32 if precision else lma.LMA_GEMM_SPLIT_BF16)
    for o_lat, o_det, f in ((lat, lma.detectors([(0.0, 0.01)]), path), (other_prec, det, path),
                            (lat, det, cut), (lat, det, junk), (lat, det, str(tmp_path / "missing.basis"))):
        c = lma.Plan(opt, o_lat, o_det)
        with pytest.raises(lma.LmaError) as e:
            c.load_basis(f)
        assert e.value.status == _lib.LMA_ERR_ARG
        with pytest.raises(lma.LmaError) as e:
            c.probe_image()                               # still no basis
        assert e.value.status == _lib.LMA_ERR_STATE
        c.close()


def _specimens():
    """Three specimens: the tiny workload, the tiny geometry with another potential, and a
    256^2 grid; each with an edited potential (a raised 12 x 12-pixel patch)."""
    import torch
    w = WORKLOADS["tiny"]
    lam, sig = lma.electron_constants(w.kv)
    out = []
    for k, n in enumerate((128, 128, 256)):
        l = n * 0.1
        opt = lma.optics(n, n, l, l, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3)
        scan = (n // 8, n // 8)
        lat = lma.lattice(scan[0], scan[1], n // 4, n // 4, 1, (0.5, 0.5), 36)
        det = lma.detectors(PAPER_RINGS)
        if k == 0:
            v = potential_slices(w, 0)
        else:
            v = np.random.default_rng(100 + k).uniform(0, 40, size=(6, n, n)).astype(np.float32)
        v_new = v.copy()
        x0, y0 = 20 + 7 * k, 30 + 5 * k
        v_new[:, y0:y0 + 12, x0:x0 + 12] += 15.0
        out.append(dict(opt=opt, lat=lat, det=det, v=v, vd=torch.from_numpy(v).cuda(), v_new=v_new,
                        bbox=(x0, y0, x0 + 12, y0 + 12), shape=(len(PAPER_RINGS), scan[1], scan[0])))
    return out


def _run(server, specs, mixed):
    """Build, LMA image, local edit and plain image for every specimen; returns the images."""
    import torch
    res = []
    reqs = []
    for k, s in enumerate(specs):
        r = dict(lma=torch.zeros(s["shape"], dtype=torch.float64, device="cuda"),
                 plain=torch.zeros(s["shape"], dtype=torch.float64, device="cuda"),
                 edit=np.zeros(s["shape"]))
        res.append(r)
        reqs.append([lambda k=k, s=s: server.build(k, s["opt"], s["lat"], s["det"], s["v"].shape[0]),
                     lambda k=k, s=s, r=r: server.image(k, s["vd"], r["lma"]),
                     lambda k=k, s=s, r=r: server.edit(k, s["v_new"], s["bbox"], 1.5, r["edit"]),
                     lambda k=k, s=s, r=r: server.plain(k, s["vd"], r["plain"])])
    if mixed:
        tickets = [reqs[k][j]() for j in range(4) for k in range(len(specs))]
        for t in tickets:
            server.wait(t)
    else:
        for k in range(len(specs)):
            for j in range(4):
                server.wait(reqs[k][j]())
    torch.cuda.synchronize()
    return [{key: (val.cpu().numpy() if hasattr(val, "cpu") else val) for key, val in r.items()} for r in res]


def test_same_results_alone_and_in_the_mix():
    specs = _specimens()
    say("serving: alone (one slot, one request at a time)")
    with lma.Server(1, 3, 1 << 36) as s:
        alone = _run(s, specs, mixed=False)
    say("serving: in the mix (three slots, every request queued at once)")
    with lma.Server(3, 3, 1 << 36) as s:
        mix = _run(s, specs, mixed=True)
    for k in range(len(specs)):
        for key in ("lma", "plain", "edit"):
            a, b = alone[k][key], mix[k][key]
            assert np.any(a != 0), (k, key)
            # identical waves and contraction tiles; only the order of FP64 atomic adds differs
            assert np.allclose(a, b, rtol=1e-12, atol=0), (k, key)
    # and the same as the plan API on the caller's stream
    s0 = specs[0]
    with lma.Plan(s0["opt"], s0["lat"], s0["det"]) as p:
        p.propagate(s0["vd"])
        direct = p.probe_image()
    assert np.allclose(alone[0]["lma"], direct, rtol=1e-12, atol=0)
    # and the served results of the tiny specimen against the FP64 oracle: its LMA image, its
    # plain image, and the local edit (the oracle re-propagating the translates within the
    # radius with the edited potential and re-forming the probes that use them; the request
    # patches those probes into a zero image)
    from oracle.lma import LMA, recompute_sets
    from oracle.multislice import plain_image
    w = WORKLOADS["tiny"]
    st = oracle_setup(w, detectors=PAPER_RINGS)
    ol = oracle_lattice(w, st, L=36)
    om = LMA(st, ol)
    allt = [(t % ol.Rfx, t // ol.Rfx) for t in range(ol.n_translates)]
    say("serving: oracle LMA, plain and edit of the tiny specimen")
    b0 = om.propagate(s0["v"], allt)
    R, Pp = recompute_sets(ol, s0["bbox"], 1.5)
    mixed = dict(b0)
    mixed.update(om.propagate(s0["v_new"], sorted(R)))
    ref_edit = np.zeros(s0["shape"])
    img_edit = om.image(s0["v_new"], basis=mixed)
    for a, b in Pp:
        ref_edit[:, b, a] = img_edit[:, b, a]
    for key, ref in (("lma", om.image(s0["v"], basis=b0)), ("plain", plain_image(st, s0["v"])), ("edit", ref_edit)):
        e = image_errors(mix[0][key], ref, TOL32)
        say(f"  served {key} image vs oracle, per-detector rel L2 {e}")


def test_admission_by_footprint():
    specs = _specimens()[:2]
    s0 = specs[0]
    s1 = specs[1]
    need = lma.footprint(s0["opt"], s0["lat"], s0["det"], s0["v"].shape[0])
    need1 = lma.footprint(s1["opt"], s1["lat"], s1["det"], s1["v"].shape[0])
    budget = max(need, need1) + min(need, need1) // 2
    assert need + need1 > budget
    # room for one of the two specimens at a time: the second build waits for the first release
    import time
    with lma.Server(2, 2, budget) as s:
        sub = {}
        sub["b0"] = time.monotonic()
        t0 = s.build(0, s0["opt"], s0["lat"], s0["det"], s0["v"].shape[0])
        sub["b1"] = time.monotonic()
        t1 = s.build(1, s1["opt"], s1["lat"], s1["det"], s1["v"].shape[0])
        sub["r0"] = time.monotonic()
        r0 = s.release(0)
        lat0, _ = s.wait(t0)
        lat_r0, _ = s.wait(r0)
        lat1, svc1 = s.wait(t1)
        say(f"  build 0 {lat0:.1f} ms, release 0 {lat_r0:.1f} ms, build 1 {lat1:.1f} ms (service {svc1:.1f})")
        # completion times on one clock (submission taken just before each call): build 1 was
        # admitted only once the release had freed the first specimen's bytes
        done_r0 = sub["r0"] * 1e3 + lat_r0
        start_b1 = sub["b1"] * 1e3 + lat1 - svc1
        assert start_b1 >= done_r0 - 0.5
        assert s.in_use() == need1
        assert s.plan_info(1).n_rows > 0

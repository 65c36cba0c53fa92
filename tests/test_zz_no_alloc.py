"""GPU: lma_plain_image_noalloc (the plain image for callers that cannot allocate) against
lma_plain_image on the same plan, through the C ABI: two calls in a row, the second with a
smaller input, and the refusals."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import paper_2310_16829_amd as lma
from paper_2310_16829_amd import _lib
from synth import WORKLOADS, potential_slices
from tests.test_gpu_parity import PAPER_RINGS, TOL32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(w, window=(0, 0, 0, 0), nx=None, lx=None, scan=None):
    lam, sig = lma.electron_constants(w.kv)
    nx = nx or w.nx
    lx = lx or w.lx
    opt = lma.optics(nx, nx, lx, lx, lam, sig, w.dz, w.bandlimit, w.alpha_mrad * 1e-3, w.defocus, w.cs)
    scan = scan or w.scan
    lat = lma.lattice(scan[0], scan[1], nx // w.basis_px, nx // w.basis_px, 1, w.offset_frac, w.L, window=window)
    return lma.Plan(opt, lat, lma.detectors(PAPER_RINGS))


def test_plain_image_noalloc_matches_plain_image():
    import torch
    w = WORKLOADS["tiny"]
    v = torch.from_numpy(potential_slices(w, 0)).cuda()
    with _plan(w) as plan:
        shape = plan.image_shape()
        for nsl, flags, weight in ((10, 0, 1.0), (4, lma.LMA_ACCUMULATE, 0.5)):
            vs = v[:nsl].contiguous()
            say(f"noalloc: tiny workload, {nsl} slices, flags {flags}")
            base = torch.rand(shape, dtype=torch.float64, device="cuda")
            want = plan.plain_image(vs, base.clone(), flags=flags, weight=weight)
            got = plan.plain_image_noalloc(vs, base.clone(), flags=flags, weight=weight)
            torch.cuda.synchronize()
            g, r = got.cpu().numpy(), want.cpu().numpy()
            errs = [rel_l2(g[k], r[k]) for k in range(r.shape[0])]
            say("  per-detector rel L2 against lma_plain_image", errs)
            assert max(errs) < 1e-12
            assert not np.array_equal(g, base.cpu().numpy())
    # a second plan, smaller: 64^2 grid, 3 slices, a 5 x 3-probe window
    rng = np.random.default_rng(64)
    v64 = torch.from_numpy(rng.uniform(0, 40, size=(3, 64, 64)).astype(np.float32)).cuda()
    with _plan(w, window=(1, 2, 5, 3), nx=64, lx=6.4, scan=(8, 8)) as plan:
        want = plan.plain_image(v64, device=True)
        got = plan.plain_image_noalloc(v64, torch.zeros_like(want))
        torch.cuda.synchronize()
        assert rel_l2(got.cpu().numpy(), want.cpu().numpy()) < 1e-12


def test_plain_image_noalloc_refusals():
    import torch
    w = WORKLOADS["tiny"]
    with _plan(w, window=(0, 0, 2, 2)) as plan:
        v = torch.zeros((2, 128, 128), dtype=torch.float32, device="cuda")
        img = torch.zeros(plan.image_shape(), dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            plan.plain_image_noalloc(v.cpu().numpy(), img)          # host potential
        # 600 slices of 128^2 need 75 MiB of transmission tables: beyond the scratch array
        big = torch.zeros((600, 128, 128), dtype=torch.float32, device="cuda")
        with pytest.raises(lma.LmaError) as e:
            plan.plain_image_noalloc(big, img)
        assert e.value.status == _lib.LMA_ERR_ARG and "scratch" in str(e.value)

"""GPU: captured slice loops (LMA_GRAPH), the autotuner and the uneven batch (lma_batch_*).

A graph replays the kernels of an eager run with the same launch shapes, so basis rows (no
atomics) must match the eager path bit for bit and images (FP64 atomics, any order) to 1e-12;
each replay is checked, with eager work and synchronisations between replays. The eager path
itself is checked against the oracle in test_gpu_parity.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import paper_2310_16829_amd as lma
from oracle.lma import LMA
from synth import WORKLOADS, potential_slices
from tests.test_gpu_parity import TOL32, build, crop, image_errors, window_probes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _plan(w, flags=0, **kw):
    return build(w, flags=flags, **kw)


def test_graph_replays_match_eager():
    w = WORKLOADS["tiny"]
    vs = [potential_slices(w, c) for c in range(3)]
    eager, _, _ = _plan(w, batch=300)              # ragged: 1024 rows in 300-wave batches
    graph, _, _ = _plan(w, flags=lma.LMA_GRAPH, batch=300)
    assert graph.info().graphs == 0
    for rep in range(4):
        v = vs[rep % 3]
        say(f"graph replay {rep}: configuration {rep % 3}")
        eager.propagate(v)
        ref_rows = eager.basis_rows(0, eager.n_rows)
        ref_img = eager.probe_image()
        graph.propagate(v)
        assert np.array_equal(graph.basis_rows(0, graph.n_rows), ref_rows), f"replay {rep}: basis rows differ"
        assert _rel(graph.probe_image(), ref_img) < 1e-12
        ref_plain = eager.plain_image(v)
        assert _rel(graph.plain_image(v), ref_plain) < 1e-12
    i = graph.info()
    assert i.graphs == 2        # the propagation and the plain image, each captured once
    eager.close()
    graph.close()


def test_autotuned_plan_matches_oracle():
    w = WORKLOADS["tiny"]
    t = lma.autotune(128, 128)
    say("autotune 128^2:", t)
    assert t["tile_width"] in (4, 8, 16) and t["batch"] >= 64 and t["candidates"] >= 2
    assert t["us_per_wave_slice"] > 0
    assert lma.autotune(128, 128) == t                  # cached
    t2 = lma.autotune(640, 640, max_bytes=1 << 28)
    say("autotune 640^2:", t2)
    assert t2["tile_width"] in (4, 8)
    with pytest.raises(lma.LmaError):
        lma.autotune(100, 100)
    plan, st, ol = _plan(w, flags=lma.LMA_AUTOTUNE, window=(2, 3, 5, 4))
    assert plan.info().tile_width == t["tile_width"]
    v = potential_slices(w, 0)
    plan.propagate(v)
    ref = crop(LMA(st, ol).image(v, window_probes(plan)), plan)
    image_errors(plan.probe_image(), ref, TOL32)


def test_uneven_batch_matches_each_plan_alone():
    w = WORKLOADS["tiny"]
    rng = np.random.default_rng(7)
    specs = [dict(nx=96, ny=96, lx=9.6, ly=9.6, scan=(12, 12), R=(24, 24), L=9, window=(1, 2, 5, 4), batch=50),
             dict(window=(3, 3, 6, 5)),
             dict(nx=192, ny=64, lx=19.2, ly=6.4, scan=(24, 8), R=(48, 16), L=9, window=(20, 5, 4, 3)),
             dict(nx=640, ny=96, lx=64.0, ly=9.6, scan=(80, 12), R=(160, 24), L=9, window=(40, 7, 4, 3)),
             dict(window=(8, 1, 5, 6), prop_window=(64, 32))]     # translates on windows
    nsl = [3, 10, 7, 2, 10]
    pots = [potential_slices(w, 0) if i in (1, 4) else
            rng.uniform(0, 40, size=(nsl[i], s["ny"], s["nx"])).astype(np.float32) for i, s in enumerate(specs)]
    alone = [_plan(w, **s)[0] for s in specs]
    refs = []
    for p, v in zip(alone, pots):
        p.propagate(v)
        refs.append((p.basis_rows(0, p.n_rows), p.probe_image()))
    inb = [_plan(w, **s) for s in specs]
    batch = lma.Batch([p for p, _, _ in inb], nsl)
    for rep in range(3):
        say(f"uneven batch, launch {rep}")
        batch.propagate(pots)
        for i, (p, _, _) in enumerate(inb):
            assert np.array_equal(p.basis_rows(0, p.n_rows), refs[i][0]), f"launch {rep}, plan {i}: basis rows"
            assert _rel(p.probe_image(), refs[i][1]) < 1e-12
        # eager work on the plans between launches
        inb[1][0].plain_image(pots[1])
    # and against the oracle for the tiny specimen
    p, st, ol = inb[1]
    ref = crop(LMA(st, ol).image(pots[1], window_probes(p)), p)
    image_errors(p.probe_image(), ref, TOL32)
    batch.close()


def test_grouped_batch_matches_each_plan_alone():
    """lma_batch_create_grouped: plans of one length class (same grid and optics) share their row
    and column passes over one wave buffer, with different slice counts and potentials; a plan
    of another size forms a class of its own and a windowed plan runs its own slice loop. Every
    plan's basis rows equal those of the plan run alone, bit for bit (the same arithmetic per
    wave), over three launches; with a 1-byte group limit every plan runs alone."""
    w = WORKLOADS["tiny"]
    rng = np.random.default_rng(11)
    specs = [dict(window=(3, 3, 6, 5)),
             dict(window=(1, 1, 4, 4)),
             dict(window=(5, 2, 3, 3)),
             dict(nx=96, ny=96, lx=9.6, ly=9.6, scan=(12, 12), R=(24, 24), L=9, window=(1, 2, 5, 4)),
             dict(window=(8, 1, 5, 6), prop_window=(64, 32))]
    nsl = [10, 6, 10, 4, 7]
    pots = [potential_slices(w, 0),
            rng.uniform(0, 40, size=(nsl[1], 128, 128)).astype(np.float32),
            potential_slices(w, 1),
            rng.uniform(0, 40, size=(nsl[3], 96, 96)).astype(np.float32),
            potential_slices(w, 2)[:nsl[4]]]
    alone = [_plan(w, **s)[0] for s in specs]
    refs = []
    for p, v in zip(alone, pots):
        p.propagate(v)
        refs.append((p.basis_rows(0, p.n_rows), p.probe_image()))
    for limit in (0, 1):
        inb = [_plan(w, **s) for s in specs]
        batch = lma.Batch([p for p, _, _ in inb], nsl, grouped=True, max_group_bytes=limit)
        for rep in range(3):
            say(f"grouped batch (limit {limit}), launch {rep}")
            batch.propagate(pots)
            for i, (p, _, _) in enumerate(inb):
                assert np.array_equal(p.basis_rows(0, p.n_rows), refs[i][0]), f"launch {rep}, plan {i}: basis rows"
                assert _rel(p.probe_image(), refs[i][1]) < 1e-12
            inb[0][0].plain_image(pots[0])
        if limit == 0:
            p, st, ol = inb[2]
            ref = crop(LMA(st, ol).image(pots[2], window_probes(p)), p)
            image_errors(p.probe_image(), ref, TOL32)
        batch.close()

"""GPU tests of the graph-captured time loop: runs of 32 steps are recorded
once and replayed; every replay must give the same bits as launching the
steps one by one, with eager work and synchronisations between replays."""
import numpy as np
import pytest

import paper_2310_00236_amd as hw
from helpers import (acoustic_fields, assert_bitexact, elastic_fields,
                     layered_material, smooth_medium3d)

pytestmark = pytest.mark.gpu


def _plan2d(comp="twosum"):
    nx, ny = 130, 70
    rho, kappa, c = layered_material(nx, ny, 1100)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", comp, 1.0, dt, 0, 64)
    p = hw.Plan(pb)
    p.set_material([rho, kappa])
    p.set_fields(acoustic_fields(nx, ny, 1101, "f16"))
    return p


def test_graph_replays_match_single_launches():
    graphed = _plan2d()
    eager = _plan2d()
    for rep in range(4):
        graphed.advance(70)               # 1 aligning step? no: 2 graph runs + 6
        for _ in range(70):
            eager.advance(1)              # never captured
        a = graphed.get_fields(comps=True)
        b = eager.get_fields(comps=True)
        assert_bitexact(a[0], b[0], f"replay {rep}")
        assert_bitexact(a[1], b[1], f"replay {rep} comps")
        eager.record_energy()             # eager work between replays
        graphed.advance(1)                # odd count: next run starts misaligned
        eager.advance(1)
    for p in (graphed, eager):
        p.close()


def test_batch_graph_matches_single_launches():
    def mk():
        out = []
        for i, (nx, ny) in enumerate([(90, 60), (64, 64), (200, 33)]):
            rho, kappa, c = layered_material(nx, ny, 1200 + i)
            dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
            pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum", 1.0, dt, 0, 64)
            p = hw.Plan(pb)
            p.set_material([rho, kappa])
            p.set_fields(acoustic_fields(nx, ny, 1300 + i, "f16"))
            out.append(p)
        rho, lam, mu, cp = smooth_medium3d(12, 10, 9, 1400)
        pb = hw.Problem("elastic3d", 12, 10, 9, 2, "f16", "twosum", 1.0,
                        0.4 * hw.cfl_bound("elastic3d", 2) / cp, 0, 64)
        p = hw.Plan(pb)
        p.set_material([rho, lam, mu])
        p.set_fields(elastic_fields(12, 10, 9, 1401))
        out.append(p)
        return out

    steps = [150, 97, 203, 130]
    batch = mk()
    for _ in range(2):
        hw.batch_advance(batch, steps, energy_every=50)
    eager = mk()
    for p, n in zip(eager, steps):
        for _ in range(2):
            for _ in range(n):
                p.advance(1, 50)
    for a, b in zip(batch, eager):
        fa, ca = a.get_fields(comps=True)
        fb, cb = b.get_fields(comps=True)
        assert_bitexact(fa, fb, "batch graph")
        assert_bitexact(ca, cb, "batch graph comps")
        ea, sa = a.energy_trace()
        eb, sb = b.energy_trace()
        assert np.array_equal(sa, sb) and np.array_equal(ea, eb)
    for p in batch + eager:
        p.close()

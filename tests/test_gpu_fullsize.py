"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times: the 512^3 elastic workload in its tuned (fused) kernel
shape, checked cell by cell on sampled cells against the oracle on local
periodic patches; and the 64-shot batched workload, every shot
bit-identical batched and alone."""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from paper_2310_00236_amd import tuning

pytestmark = pytest.mark.gpu

FIELDS = oracle.ELASTIC_FIELDS


def _decode_state(plan, blob):
    """Split an fp16 + compensation state blob into per-field value and
    compensation arrays [nz, ny, nx] (the blob holds each field's padded
    words, (value, compensation) side by side, after a fixed header)."""
    pb = plan.pb
    pitch = (pb.nx + 63) // 64 * 64
    n = pitch * pb.ny * pb.nz
    field_bytes = (n * 4 + 255) // 256 * 256
    head = len(blob) - len(FIELDS) * field_bytes
    vals, comps = {}, {}
    for i, k in enumerate(FIELDS):
        w = np.frombuffer(blob, dtype=np.float16, count=2 * n,
                          offset=head + i * field_bytes).reshape(pb.nz, pb.ny, pitch, 2)
        vals[k] = w[:, :, :pb.nx, 0]
        comps[k] = w[:, :, :pb.nx, 1]
    return vals, comps


def test_elastic_512_sampled_one_step():
    """512^3 smooth medium, fp16 + TwoSum, the tuned kernel shape: after 20
    steps, one more step is checked on 40 sampled cells (and the corners)
    against the oracle run on 9^3 periodic patches around them (one step of
    the scheme reaches 2 cells)."""
    n = 512
    w = workloads.smooth3d(n, nsteps=20)
    pb = hw.Problem("elastic3d", n, n, n, 2, "f16", "twosum", w.dx, w.dt, 0, 0)
    plan = hw.Plan(pb)
    plan.set_tile(tuning.best_tile("elastic3d", 2, "f16", "twosum", n, n, n))
    assert hw.tiles("elastic3d")[plan_tile(plan)][3] == 2      # the fused kernel kind
    plan.set_material([w.rho, w.lam, w.mu])
    plan.set_fields(w.fields())
    plan.advance(w.nsteps)
    before = _decode_state(plan, plan.export_state())
    plan.advance(1)
    after = _decode_state(plan, plan.export_state())
    plan.close()
    rng = np.random.default_rng(9)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 255)] + \
        [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(40)]
    m = 4
    for (k, j, i) in pts:
        idx = np.ix_(np.arange(k - m, k + m + 1) % n, np.arange(j - m, j + m + 1) % n,
                     np.arange(i - m, i + m + 1) % n)
        f = {key: before[0][key][idx].astype(np.float64) for key in FIELDS}
        c = {key: before[1][key][idx].astype(np.float64) for key in FIELDS}
        s = 2 * m + 1
        o, oc, _ = oracle.elastic3d(s, s, s, w.dx, w.dt, w.rho[idx], w.lam[idx],
                                    w.mu[idx], f, storage="f16", stencil="f32",
                                    comp="twosum", comps=c, nsteps=1)
        for key in FIELDS:
            assert float(after[0][key][k, j, i]) == o[key][m, m, m], (key, k, j, i)
            assert float(after[1][key][k, j, i]) == oc[key][m, m, m], (key, k, j, i)


def plan_tile(plan):
    return tuning.best_tile("elastic3d", 2, plan.pb.storage, plan.pb.comp,
                            plan.pb.nx, plan.pb.ny, plan.pb.nz)


def test_batched_64_shot_workload_equals_solo_runs():
    """The benchmark's 64 layered shots (sides 256..2048, 500..5000 steps,
    fp16 + TwoSum, tuned tiles): batched launches and one shot at a time end
    in byte-identical states."""
    t0 = time.time()

    def note(msg):
        print(f"# {time.time() - t0:7.1f} s  {msg}", file=sys.stderr, flush=True)

    sizes = workloads.shot_sizes(64)
    shots = [workloads.shot(nx, ny, ns, i) for i, (nx, ny, ns) in enumerate(sizes)]
    note("shots generated")

    def make():
        plans = []
        for s in shots:
            pb = hw.Problem("acoustic2d", s.nx, s.ny, 1, 4, "f16", "twosum",
                            s.dx, s.dt, 0, 0)
            p = hw.Plan(pb)
            p.set_tile(tuning.best_tile("acoustic2d", 4, "f16", "twosum", s.nx, s.ny))
            p.set_material([s.rho, s.kappa])
            p.set_fields(s.fields())
            plans.append(p)
        return plans

    batched = make()
    note("batched plans ready")
    hw.batch_advance(batched, [s.nsteps for s in shots])
    blobs = [p.export_state() for p in batched]
    for p in batched:
        p.close()
    note("batched run exported")
    for i, (s, blob) in enumerate(zip(shots, blobs)):
        pb = hw.Problem("acoustic2d", s.nx, s.ny, 1, 4, "f16", "twosum", s.dx, s.dt, 0, 0)
        p = hw.Plan(pb)
        p.set_tile(tuning.best_tile("acoustic2d", 4, "f16", "twosum", s.nx, s.ny))
        p.set_material([s.rho, s.kappa])
        p.set_fields(s.fields())
        p.advance(s.nsteps)
        same = p.export_state() == blob        # a bool: no diff of the bytes
        assert same, s.name
        p.close()
        if i % 8 == 7:
            note(f"{i + 1} solo runs match")

"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times: the 512^3 elastic workload in its tuned (fused) kernel
shape, checked cell by cell against the oracle on whole planes around the
kernel's z-segment boundaries and on patches around random cells; and the
64-shot batched workload, every shot bit-identical batched and alone."""
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
    """Split a state blob into per-field value and compensation arrays
    [nz, ny, nx] (the blob holds each field's padded words after a fixed
    header: fp32 values, or (fp16 value, fp16 compensation) side by side)."""
    pb = plan.pb
    pitch = (pb.nx + 63) // 64 * 64
    n = pitch * pb.ny * pb.nz
    comp = pb.comp != "none"
    words = 2 if comp else 1
    dt = np.float32 if pb.storage == "f32" else np.float16
    esz = np.dtype(dt).itemsize
    field_bytes = (n * esz * words + 255) // 256 * 256
    head = len(blob) - len(FIELDS) * field_bytes
    vals, comps = {}, {}
    for i, k in enumerate(FIELDS):
        w = np.frombuffer(blob, dtype=dt, count=words * n,
                          offset=head + i * field_bytes).reshape(pb.nz, pb.ny, pitch, words)
        vals[k] = w[:, :, :pb.nx, 0]
        comps[k] = w[:, :, :pb.nx, 1] if comp else None
    return vals, comps


def _segment_planes(tile, n):
    """z planes where the tuned fused kernel's segments meet (a segment of
    tz planes starts with warm-up planes whose velocities it recomputes)."""
    tz = hw.tiles("elastic3d")[tile][2]
    return sorted({(b + d) % n for b in range(0, n, tz) for d in (-1, 0)})


@pytest.mark.parametrize("storage,comp", [("f16", "twosum"), ("f32", "none")])
def test_elastic_512_one_step_on_segment_boundary_slabs(storage, comp):
    """512^3 smooth medium in the tuned (fused, z-marching) kernel shape, as
    the benchmark times it: after 20 steps, one more step is compared with
    the oracle on whole planes -- the five planes around every boundary
    between the kernel's z segments (wrap-around included), so every column
    edge (x = 63/64, y where the 64 x ty columns meet) of every segment's
    warm-up and last planes -- and on 9^3 patches around 40 random cells.
    The oracle runs periodic slabs of 9 planes; the middle five depend only
    on planes inside the slab (one step reaches two cells)."""
    n = 512
    w = workloads.smooth3d(n, nsteps=20)
    pb = hw.Problem("elastic3d", n, n, n, 2, storage, comp, w.dx, w.dt, 0, 0)
    plan = hw.Plan(pb)
    tile = tuning.best_tile("elastic3d", 2, storage, comp, n, n, n)
    plan.set_tile(tile)
    assert hw.tiles("elastic3d")[tile][3] == 2      # the fused kernel kind
    plan.set_material([w.rho, w.lam, w.mu])
    plan.set_fields(w.fields())
    plan.advance(w.nsteps)
    before = _decode_state(plan, plan.export_state())
    plan.advance(1)
    after = _decode_state(plan, plan.export_state())
    plan.close()

    def check(kidx, jidx, iidx, centre, local, label):
        """Run the oracle on the periodic patch kidx x jidx x iidx of the
        state and compare the GPU's cells `centre` (global index arrays per
        axis) with the oracle's cells `local` (patch index arrays)."""
        idx = np.ix_(kidx, jidx, iidx)
        f = {key: before[0][key][idx].astype(np.float64) for key in FIELDS}
        c = {key: before[1][key][idx].astype(np.float64) for key in FIELDS} \
            if comp != "none" else None
        o, oc, _ = oracle.elastic3d(len(iidx), len(jidx), len(kidx), w.dx, w.dt,
                                    w.rho[idx], w.lam[idx], w.mu[idx], f,
                                    storage=storage, stencil="f32", comp=comp,
                                    comps=c, nsteps=1)
        for key in FIELDS:
            got = after[0][key][np.ix_(*centre)].astype(np.float64)
            want = o[key][np.ix_(*local)]
            assert np.array_equal(got, want) and \
                np.array_equal(np.signbit(got), np.signbit(want)), (key, label)
            if comp != "none":
                got = after[1][key][np.ix_(*centre)].astype(np.float64)
                want = oc[key][np.ix_(*local)]
                assert np.array_equal(got, want) and \
                    np.array_equal(np.signbit(got), np.signbit(want)), ("comp", key, label)

    full = np.arange(n)
    done = set()
    for k0 in _segment_planes(tile, n):
        if k0 in done:
            continue
        kidx = np.arange(k0 - 4, k0 + 5) % n
        mid = kidx[2:7]
        done.update(int(k) for k in mid)
        check(kidx, full, full, (mid, full, full), (np.arange(2, 7), full, full),
              f"planes {list(mid)}")
    rng = np.random.default_rng(9)
    m = 4
    one = np.array([m])
    for _ in range(40):
        k, j, i = (int(v) for v in rng.integers(0, n, size=3))
        ax = [np.arange(c - m, c + m + 1) % n for c in (k, j, i)]
        check(*ax, (np.array([k]), np.array([j]), np.array([i])), (one, one, one),
              f"cell {(k, j, i)}")


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

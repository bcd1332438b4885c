"""Host-side checks of the benchmark's reproduction sections (Sec. 3 and
App. A): with a stand-in plan that returns arrays of the right shapes, the
sections run for full and shortened step counts and report every field of
their JSON, comparisons with the stored FP64 references included.  No GPU:
timings are fixed and the traces random; only the bookkeeping is checked."""
import types

import numpy as np
import pytest

import bench
import paper_2310_00236_amd as hw


class _Event:
    def __init__(self, **_):
        pass

    def record(self, stream=None):
        pass

    def elapsed_time(self, other):
        return 10.0


_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
    synchronize=lambda: None, Event=_Event, current_stream=lambda: None))


class _Plan:
    """Records the calls a benchmark section makes; returns traces of the
    documented shapes."""

    def __init__(self, pb):
        self.pb, self.n, self.every, self.nrec = pb, 0, 0, 0
        self.rng = np.random.default_rng(0)
        self.extra = []           # steps of explicit record_energy calls

    @property
    def step(self):
        return self.n

    def record_energy(self):
        self.extra.append(self.n)

    def set_tile(self, tile):
        assert 0 <= tile < len(hw.tiles(self.pb.physics))

    def set_material(self, m):
        assert len(m) == (2 if self.pb.physics == "acoustic2d" else 3)

    def set_fields(self, f):
        pass

    def set_source(self, ix, iy, samples):
        assert len(samples) <= self.pb.src_cap

    def set_receivers(self, cells):
        self.nrec = len(cells)

    def advance(self, n, every=0):
        self.n += n
        self.every = every

    def receiver_trace(self):
        m = 5 if self.pb.physics == "elastic2d" else 3
        return self.rng.normal(size=(min(self.n, self.pb.rec_steps), self.nrec, m))

    def energy_trace(self):
        steps = np.arange(0, self.n + 1, self.every) if self.every else np.zeros(0, int)
        steps = np.sort(np.concatenate([steps, np.array(self.extra, dtype=int)]))
        if len(steps) == 0:
            steps = np.zeros(1, int)
        return 1.0 + 1e-4 * self.rng.random(len(steps)), steps

    def close(self):
        pass


_hw = types.SimpleNamespace(Problem=hw.Problem, Plan=_Plan, tiles=hw.tiles,
                            tile_label=hw.tile_label)


@pytest.mark.parametrize("nsteps", [3000, 60000])
def test_app_a_section(nsteps):
    r = bench.run_app_a(_hw, _torch, nsteps, big=64, big_steps=4)
    assert r["reference"] == "FP64 oracle"
    assert set(r["variants"]) == {f"{s}+{c}" for s, c in bench.APP_A_VARIANTS}
    for v in r["variants"].values():
        assert {"glups", "ms_total", "tile", "energy_change_after_source",
                "vy_trace_rel_l2_vs_fp64", "energy_max_rel_dev_vs_fp64"} <= set(v)
        # the source fires for 4801 steps: no post-source change before that
        assert (v["energy_change_after_source"] is None) == (nsteps < 6000)
    assert set(r["throughput_64"]) == {"f32+none", "f16+twosum", "f16+none"}


@pytest.mark.parametrize("nsteps", [3000, 60000])
def test_paper_section(nsteps):
    r = bench.run_paper(_hw, _torch, nsteps)
    assert r["reference"] == "FP64 oracle"
    assert len(r["variants"]) == len(bench.PAPER_VARIANTS)
    for v in r["variants"].values():
        assert {"glups", "ms_total", "p_trace_rel_l2_vs_fp64",
                "energy_max_rel_dev_vs_fp64"} <= set(v)
    assert "discretisation_rel_l2_ppw10_vs_ppw30" in r


def test_trace_comparison_covers_only_the_steps_run():
    gold = {"steps": np.array([50, 100, 150]),
            "rec": np.array([[0.0], [2.0], [4.0]])}
    trace = np.zeros(120)
    trace[99] = 2.0
    assert bench.trace_rel_l2(trace, gold, 0) == 0.0      # rows 50 and 100 only
    assert bench.trace_rel_l2(np.zeros(60), gold, 0) is None   # reference still zero


def test_window_drift_needs_two_samples():
    e = np.array([1.0, 1.5, 0.5, 2.0])
    st = np.array([0, 10, 20, 30])
    assert bench.window_drift(e, st, 10, 20) == pytest.approx(2 / 3)
    assert bench.window_drift(e, st, 5, 15) is None
    assert bench.window_drift(e, st, 0, 30) == pytest.approx(1.0)


def test_short_timed_window_still_has_its_drift():
    """A 20-step timed run (no energy step inside it) reports the drift
    between the energies at its two ends, not a vacuous 0."""
    import workloads
    w = workloads.layered2d(64, nsteps=20)
    r = bench.run_variant(_hw, _torch, w, "f16", "twosum", 20, 5, 0)
    assert r["energy_samples_window"] == 2
    assert r["energy_drift_window"] is not None and r["energy_drift_window"] > 0


def test_drift_run_against_the_fp64_record():
    import workloads
    w = workloads.layered2d(64, nsteps=3000)
    ref = {0: 1.0, 1000: 1.0 + 1e-13}
    r = bench.drift_run(_hw, w, "f16", "twosum", 0, 3000, ref)
    assert r["steps"] == 3000 and r["energy_samples"] == 4
    assert r["fp64_reference_steps"] == [0, 1000]
    assert 0 < r["energy_drift_vs_fp64"] < 1e-3
    assert bench.drift_run(_hw, w, "f16", "twosum", 0, 3000, None)[
        "energy_drift_vs_fp64"] is None


def test_layered_fp64_record_matches_the_oracle():
    """The stored FP64 energies of the 4096^2 layered workload: step 0 is
    the oracle's energy of the start rounded to each format, and the FP64
    run conserves it (relative 1e-12) at every stored step."""
    import oracle
    import workloads
    gold = bench.read_layered_golden()
    assert {"f16", "f32", "bf16"} <= set(gold)
    w = workloads.layered2d(nsteps=10000)
    for start, rec in gold.items():
        f = {k: oracle.round_to(v, start) for k, v in w.fields().items()}
        e0 = oracle.acoustic2d_energy(w.nx, w.ny, w.order, w.dx, w.dt, w.rho, w.kappa, f)
        assert rec[0] == pytest.approx(e0, rel=1e-14, abs=0)
        for n, e in rec.items():
            assert abs(e - rec[0]) <= 1e-12 * rec[0], (start, n)

"""Seeded random cases of the 2D acoustic step on the two-steps-per-launch
shapes against the oracle: grid sizes from one cell to several tiles in
each direction, both orders, every storage format and update (8-bit words
included), odd and even step counts, energy logs at odd intervals, and half
of the cases with a point source and receivers at random cells.  Fields,
compensation terms, receiver traces and energies must be the oracle's, bit
for bit (energies to 1e-12)."""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from helpers import acoustic_fields, assert_bitexact, layered_material

pytestmark = pytest.mark.gpu

TWO = [t for t, s in enumerate(hw.tiles("acoustic2d")) if s[2] == 2]
COMBOS = [("f32", "none"), ("f32", "twosum"), ("f16", "none"), ("f16", "fast2sum"),
          ("f16", "twosum"), ("f16", "twosum8"), ("bf16", "none"), ("bf16", "twosum"),
          ("bf16", "twosum8")]


def _cases(n=24, seed=20261203):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx = int(rng.choice([1, 2, 7, 63, 64, 65, 130, 200, 257, 320]))
        ny = int(rng.choice([1, 3, 16, 23, 24, 25, 48, 97, 150]))
        storage, comp = COMBOS[int(rng.integers(len(COMBOS)))]
        out.append(dict(
            nx=nx, ny=ny, order=int(rng.choice([2, 4])), storage=storage, comp=comp,
            tile=int(rng.choice(TWO)), nsteps=int(rng.integers(1, 14)),
            every=int(rng.choice([0, 3, 4])), forced=bool(rng.integers(2)),
            src=(int(rng.integers(nx)), int(rng.integers(ny))),
            recs=[(int(rng.integers(nx)), int(rng.integers(ny))) for _ in range(3)],
            seed=int(rng.integers(1 << 20))))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: (
    f"{c['nx']}x{c['ny']}-o{c['order']}-{c['storage']}-{c['comp']}-t{c['tile']}"
    f"-n{c['nsteps']}-e{c['every']}{'-src' if c['forced'] else ''}"))
def test_random_case(case):
    nx, ny, order = case["nx"], case["ny"], case["order"]
    storage, comp, n, every = case["storage"], case["comp"], case["nsteps"], case["every"]
    rho, kappa, c = layered_material(nx, ny, case["seed"])
    dt = 0.45 * hw.cfl_bound("acoustic2d", order) / c
    f = acoustic_fields(nx, ny, case["seed"] + 1, storage)
    samples = 0.5 * workloads.ricker((np.arange(n) + 0.5) * dt - 1.0, 1.0)
    forced = case["forced"]
    recs = case["recs"] if forced else []
    pb = hw.Problem("acoustic2d", nx, ny, 1, order, storage, comp, 1.0, dt, 0,
                    (n // every + 2) if every else 0,
                    src_cap=n if forced else 0, rec_cap=len(recs),
                    rec_steps=n if forced else 0)
    plan = hw.Plan(pb)
    plan.set_tile(case["tile"])
    plan.set_material([rho, kappa])
    plan.set_fields(f)
    if forced:
        plan.set_source(case["src"][0], case["src"][1], samples)
        plan.set_receivers(recs)
    plan.advance(n, every)
    g, gc = plan.get_fields(comps=True)
    trace = plan.receiver_trace() if forced else None
    energy = plan.energy_trace()[0] if every else None
    plan.close()

    fr = {k: oracle.round_to(v, storage) for k, v in f.items()}
    ref = oracle.acoustic2d(
        nx, ny, order, 1.0, dt, rho, kappa, fr, storage=storage, stencil="f32", comp=comp,
        nsteps=n, energy_every=every,
        source=(case["src"][0], case["src"][1], samples) if forced else None,
        receivers=recs if forced else None)
    w, wc, we = ref[:3]
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    if forced:
        assert np.array_equal(trace, ref[3]), np.argwhere(trace != ref[3])[:5]
    if every:
        np.testing.assert_allclose(energy, we, rtol=1e-12, atol=0)

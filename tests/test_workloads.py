"""The seeded input generators of the batched and served configurations follow
their stated recipe (no GPU): grid sides log-uniform in [32, 512] (batch) and
[64, 2048] (serving), step counts log-uniform in [50, 2000], Poisson arrivals,
free-stream Mach uniform in [0.001, 20] at a random angle, 1-5 Gaussian bumps of
1-20 % amplitude, positive states, and the same inputs for the same seed."""
import math

import numpy as np

import workloads


def prim(q, g=1.4):
    rho = q[0]
    u, v = q[1] / rho, q[2] / rho
    return rho, u, v, (g - 1) * (q[3] - 0.5 * rho * (u * u + v * v))


def test_bump_spec_ranges():
    rng = np.random.Generator(np.random.PCG64(7))
    specs = [workloads.bump_spec(rng) for _ in range(2000)]
    mach = np.array([s["mach"] for s in specs])
    assert mach.min() >= 0.001 and mach.max() <= 20.0 and abs(mach.mean() - 10.0) < 0.5
    nb = np.array([len(s["bumps"]) for s in specs])
    assert nb.min() == 1 and nb.max() == 5
    b = np.array([bb for s in specs for bb in s["bumps"]])
    cx, cy, sig, amp, target = b.T
    assert 0 <= cx.min() and cx.max() <= 1 and 0 <= cy.min() and cy.max() <= 1
    assert 0.03 <= sig.min() and sig.max() <= 0.1
    assert 0.01 <= np.abs(amp).min() and np.abs(amp).max() <= 0.2 and (amp < 0).any() and (amp > 0).any()
    assert set(target.astype(int)) == {0, 1, 2}


def test_batch_family_recipe():
    a = workloads.batch_family(256, nsteps=200)
    b = workloads.batch_family(256, nsteps=200)
    sides = np.array([c.nx for c in a])
    assert len(a) == 256 and all(c.nx == c.ny for c in a)
    assert sides.min() >= 32 and sides.max() <= 512
    # log-uniform: mean of ln(side) near (ln 32 + ln 512) / 2
    assert abs(np.log(sides).mean() - 0.5 * (math.log(32) + math.log(512))) < 0.15
    total = int((sides ** 2).sum())
    assert 9_000_000 < total < 15_000_000  # expectation about 12.05 M cells
    for ca, cb in zip(a[:16], b[:16]):
        assert ca.nx == cb.nx and np.array_equal(ca.q0, cb.q0) and ca.params == cb.params
        rho, u, v, p = prim(ca.q0)
        assert rho.min() > 0 and p.min() > 0
        assert ca.params["time_scheme"] == 1 and ca.params["order"] == 2 and ca.nsteps == 200
        assert ca.bc == (workloads.PERIODIC,) * 4 and ca.dx == 1.0 / ca.nx
        mach = float(np.sqrt(u * u + v * v).max())  # c = 1 in the free stream
        assert 0.0009 < mach < 25.0
    assert sum(1 for c in a[:16] if c.nx != a[0].nx) > 0


def test_serving_trace_recipe():
    tr = workloads.serving_trace(100.0, 100.0)
    assert tr == workloads.serving_trace(100.0, 100.0)
    t = np.array([r["arrival_s"] for r in tr])
    n = np.array([r["n"] for r in tr])
    s = np.array([r["steps"] for r in tr])
    assert np.all(np.diff(t) > 0) and t.max() <= 100.0
    # Poisson at 100/s: about 10 000 arrivals, exponential gaps of mean 10 ms
    assert 9500 < len(tr) < 10500 and abs(np.diff(t).mean() - 0.01) < 0.0005
    gaps = np.diff(t)
    assert abs(np.std(gaps) / np.mean(gaps) - 1.0) < 0.05
    assert n.min() >= 64 and n.max() <= 2048 and s.min() >= 50 and s.max() <= 2000
    assert abs(np.log(n).mean() - 0.5 * (math.log(64) + math.log(2048))) < 0.05
    assert abs(np.log(s).mean() - 0.5 * (math.log(50) + math.log(2000))) < 0.05

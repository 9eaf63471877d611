"""The oracle's branch record (the limiter and HLL decisions of a step), which
the limited-map finite-difference checks of the adjoint rely on.

* Recording does not change the step.
* A smooth state's limiter is idle almost everywhere; a jump activates it in
  the cells next to the jump.
* On the batched-instance recipe, along directions where no limiter decision
  and no HLL region switches inside +-eps v over four steps, the central
  difference (eps 1e-6) of the loss equals the oracle's exact directional
  derivative (dual numbers, the branch taken) to 1e-6; directions with such
  switches show errors far above that, which is why the check needs the record.
"""
import numpy as np

import workloads as W

G53 = 5.0 / 3.0
BOX = ((0.0, 0.0), (1.0, 1.0))


def test_record_leaves_step_unchanged_and_marks_jumps(oracle):
    n = (24, 20)
    U = W.random_p1_state(n, *BOX, G53, seed=4, amp=0.05)
    m = oracle.Mesh.cartesian(n, *BOX)
    dt = oracle.cfl_dt(m, U, G53, 0.3)
    out, codes = oracle.step_branches(m, U, dt, G53, True)
    assert np.array_equal(out, oracle.step(m, U, dt, G53, True))
    assert codes.shape == (2, 480, 12)
    smooth_active = (codes[0, :, :4] != 0).mean()
    # a density jump along x = 1/2: the limiter acts next to it
    V = U.reshape(12, 20, 24).copy()
    V[0, :, 12:] *= 1.5
    V[1, :, 11:13] += 3.0  # steep slopes at the jump
    out, codes = oracle.step_branches(m, V.reshape(-1), dt * 0.5, G53, True)
    near = codes[0].reshape(20, 24, 12)[:, 10:14, 0]
    assert (near != 0).mean() > 0.5 > smooth_active
    # HLL: subsonic faces are inside the fan (code bit 1)
    assert np.all(codes[:, :, 4:] & 1)


def test_kink_free_directions_match_exact_derivative(oracle):
    N = 64
    U0 = W.batched_state(N, 2005)
    T = W.batched_state(N, 3005)[:N * N]
    m = oracle.Mesh.cartesian((N, N), *BOX)
    dts, U = [], U0
    for _ in range(4):
        dt = oracle.cfl_dt(m, U, G53, 0.3)
        dts.append(dt)
        U = oracle.step(m, U, dt, G53, True)
    vol = 1.0 / (N * N)

    def loss(U):
        for dt in dts:
            U = oracle.step(m, U, dt, G53, True)
        return 0.5 * vol * ((U[:N * N] - T) ** 2).sum()

    def path(U):
        codes = []
        for dt in dts:
            U, c = oracle.step_branches(m, U, dt, G53, True)
            codes.append(c)
        return codes

    base = path(U0)
    U0h = U0.reshape(12, N, N)
    clean, kinked = [], []
    for seed in range(4005, 4015):
        rng = np.random.default_rng(seed)
        i0, j0 = rng.integers(0, N - 6, 2)
        v = np.zeros((12, N, N))
        v[:, j0:j0 + 6, i0:i0 + 6] = rng.standard_normal((12, 6, 6))
        v = (v * np.abs(U0h)).reshape(-1)
        kinks = 0
        for sgn in (1.0, -1.0):
            for c0, c1 in zip(base, path(U0 + sgn * 1e-6 * v)):
                kinks += int((c0[:, :, :4] != c1[:, :, :4]).sum())
                kinks += int(((c0[:, :, 4:] & 3) != (c1[:, :, 4:] & 3)).sum())
        U, dU = U0.copy(), v.copy()
        for dt in dts:
            U, dU = oracle.step_jvp(m, U, dU, dt, G53, True)
        g = vol * ((U[:N * N] - T) * dU[:N * N]).sum()
        fd = (loss(U0 + 1e-6 * v) - loss(U0 - 1e-6 * v)) / 2e-6
        (kinked if kinks else clean).append(abs(fd - g) / abs(g))
    assert clean and max(clean) < 1e-6, clean
    assert kinked and max(kinked) > 1e-5, kinked

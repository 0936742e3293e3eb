"""Pins of the oracle's velocity refresh and its cadence (Sec. 4.4, Appendix D): the truncation error
d(k) against the masked integrating factor applied by brute force, its closed forms, the monotone
cadence, and the refresh leaving a velocity whose vorticity lies inside the support unchanged."""
import math

import numpy as np
import pytest
from scipy.special import ive

from oracle import ifherk, intfac, refresh, stencils


@pytest.mark.parametrize("alpha", [0.05, 0.4, 1.5])
def test_trunc_error_is_the_masked_deficit(alpha):
    """M E(a) M applied to 1 on a box is, at every point, the product over the axes of
    1 - d(i + 1) - d(n - i) (the kernel mass beyond the near and the far face): the brute-force 3D
    sum of the masked integrating factor fixes both the sum and its index convention."""
    shape = (9, 11, 13)  # nz, ny, nx
    got = intfac.apply(np.ones(shape), alpha)
    f = [np.array([1.0 - refresh.trunc_error(alpha, i + 1) - refresh.trunc_error(alpha, n - i) for i in range(n)])
         for n in shape]
    expect = f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    assert np.abs(got - expect).max() < 2e-14


def test_trunc_error_closed_forms():
    for a in (1e-3, 0.1, 2.0, 30.0):
        # kernel mass is 1 and symmetric: the tail beyond the centre is (1 - w_0) / 2
        assert abs(refresh.trunc_error(a, 1) - 0.5 * (1.0 - ive(0, 2 * a))) < 1e-15
    # small a: the leading term of e^{-2a} I_k(2a) is a^k / k!
    a = 1e-4
    for k in (1, 2, 5):
        assert abs(refresh.trunc_error(a, k) / (a ** k / math.factorial(k)) - 1.0) < 3 * a
    # large a: the difference of two Poisson(a) variables is nearly Gaussian with variance 2a
    a = 200.0
    for k in (5, 20, 40):
        gauss = 0.5 * math.erfc((k - 0.5) / math.sqrt(4 * a))
        assert abs(refresh.trunc_error(a, k) - gauss) < 2e-3 * gauss
    assert refresh.trunc_error(0.0, 3) == 0.0
    with pytest.raises(ValueError):
        refresh.trunc_error(0.1, 0)


def test_refresh_interval_is_the_last_step_within_eps():
    beta, n_buf, umax = 0.05, 4, 0.7
    for eps in (1e-8, 1e-7, 1e-5):
        q = refresh.refresh_interval(beta, n_buf, umax, eps)
        assert q >= 1
        assert refresh.estimate(beta, q, n_buf, umax) <= eps < refresh.estimate(beta, q + 1, n_buf, umax)
    # tighter eps or a thinner buffer never allows more steps
    qs = [refresh.refresh_interval(beta, n_buf, umax, e) for e in (1e-5, 1e-7, 1e-8)]
    assert qs[0] >= qs[1] >= qs[2]
    assert refresh.refresh_interval(beta, 2, umax, 1e-6) < refresh.refresh_interval(beta, 4, umax, 1e-6)
    # one step already too much, or nothing to refresh
    assert refresh.refresh_interval(beta, 0, umax, 1e-12) == 0
    assert refresh.refresh_interval(beta, n_buf, 0.0, 1e-12, q_cap=77) == 77


def test_refresh_keeps_a_velocity_with_vorticity_inside_the_support():
    """u = Vor2Vel(C f) with f compact inside the support: C u equals C f on the support (D C f = 0
    makes -C Cbar L^{-1} the identity there), so the refresh recomputes the same u."""
    n, dx, n_buf = 16, 0.4, 3
    rng = np.random.default_rng(5)
    f = np.zeros((3, n, n, n))
    f[:, 5:-5, 5:-5, 5:-5] = rng.standard_normal((3, n - 10, n - 10, n - 10))
    u = ifherk.vor2vel(stencils.curl(f, dx), dx)
    assert np.abs(refresh.velocity_refresh(u, dx, n_buf) - u).max() < 1e-12 * np.abs(u).max()
    # a velocity with vorticity outside the support changes, and the result is divergence free
    g = rng.standard_normal((3, n, n, n))
    v = refresh.velocity_refresh(g, dx, n_buf)
    assert np.abs(v - g).max() > 0.1
    assert np.abs(stencils.div(v, dx)[1:-1, 1:-1, 1:-1]).max() < 1e-11 * np.abs(v).max() / dx


def test_component_max_on_the_solution_domain():
    u = np.zeros((3, 10, 10, 10))
    u[1, 5, 5, 5] = -0.3
    u[2, 0, 5, 5] = 9.0  # outside the solution domain of n_buf = 1
    assert refresh.component_max(u, 1) == 0.3
    assert refresh.component_max(u, 0) == 9.0


def test_repeated_masked_factors_follow_the_single_factor_estimate():
    """Sec. 4.4: q masked applications of E(a) are well approximated by one masked E(q a), so the deficit
    of a uniform field a few points inside a face follows d_{q a}(k).  Brute force: at k = 5 and 7 the
    repeated deficit stays within 0 to 20 % above the estimate for q up to 6 (at the face itself, k = 1,
    the repeated truncation loses up to 40 % more)."""
    alpha, shape = 0.3, (9, 9, 40)
    h = np.ones(shape)
    for q in range(1, 7):
        h = intfac.apply(h, alpha)
        line = h[4, 4, :]
        for k in (5, 7):
            rep = (line[20] - line[k - 1]) / line[20]
            est = refresh.trunc_error(q * alpha, k)
            assert 1.0 - 1e-9 <= rep / est <= 1.2, (q, k, rep, est)


# ---- the multi-step drivers (Sec. 4.3, 4.4): control flow pinned on small boxes -------------------

def _compact_velocity(n=12, lo=5, hi=7, dx=0.3, seed=8):
    """u0 = Cbar a with a random potential on the cells [lo, hi)^3: divergence free, compact, and with
    vorticity that the integrating factors carry outwards step by step."""
    rng = np.random.default_rng(seed)
    a = np.zeros((3, n, n, n))
    a[:, lo:hi, lo:hi, lo:hi] = rng.standard_normal((3, hi - lo, hi - lo, hi - lo))
    u = stencils.curl_bar(a, dx)
    return u * (0.5 / np.abs(u).max()), dx


def test_run_refreshes_after_every_q_cap_steps():
    """With eps so large that every estimate passes, q_max = q_cap: five steps at q_cap = 2 are
    step, step, refresh, step, step, refresh, step, and the refreshes are not no-ops here."""
    u0, dx = _compact_velocity()
    dt, re, n_buf = 0.2, 100.0, 2
    u, d, nref, qs = refresh.run(u0, 5, dt, dx, re, "A", n_buf, eps=1e9, q_cap=2)
    assert nref == 2 and qs == [2, 2, 2]
    v = u0
    for k in range(1, 6):
        v, dv = ifherk.step(v, dt, dx, re, "A", n_buf=n_buf)
        if k in (2, 4):
            w = refresh.velocity_refresh(v, dx, n_buf)
            assert np.abs(w - v).max() > 1e-6 * np.abs(v).max()
            v = w
    assert np.array_equal(u, v) and np.array_equal(d, dv)


def test_run_refreshes_exactly_after_q_steps_for_eps_between_estimates():
    """eps between the estimates after q and q + 1 steps (Appendix D) gives q_max = q: q - 1 steps take
    no refresh and equal plain steps; q steps end with one refresh of the q-step velocity."""
    u0, dx = _compact_velocity(seed=9)
    dt, re, n_buf, q = 0.2, 100.0, 2, 3
    beta = dt / (dx * dx * re)
    um = refresh.component_max(u0, n_buf)
    lo, hi = refresh.estimate(beta, q, n_buf, um), refresh.estimate(beta, q + 1, n_buf, um)
    assert lo < hi
    eps = math.sqrt(lo * hi)
    plain = [u0]
    for _ in range(q):
        plain.append(ifherk.step(plain[-1], dt, dx, re, "A", n_buf=n_buf)[0])
    u, _, nref, qs = refresh.run(u0, q - 1, dt, dx, re, "A", n_buf, eps)
    assert nref == 0 and qs == [q] and np.array_equal(u, plain[q - 1])
    u, _, nref, qs = refresh.run(u0, q, dt, dx, re, "A", n_buf, eps)
    assert nref == 1 and qs[0] == q and len(qs) == 2
    assert np.array_equal(u, refresh.velocity_refresh(plain[q], dx, n_buf))
    with pytest.raises(ValueError):  # a buffer too thin for eps: no step can be taken
        refresh.run(u0, 1, dt, dx, re, "A", n_buf, eps=1e-300)


def test_run_adaptive_first_step_only_sets_the_domain():
    """The first classification sets D_supp and D_soln without re-initialising: one adaptive step is the
    plain step on the block masks of u0's weights."""
    from oracle import blocks

    u0, dx = _compact_velocity()
    dt, re, nb, n_buf = 0.2, 100.0, 3, 1
    u, d, nre, Ws, edge = refresh.run_adaptive(u0, 1, dt, dx, re, "A", n_buf, nb, 0.0, 1e-1, 0)
    mu, nu = blocks.weights(u0, dx, nb, n_buf)
    W, supp, soln, xsoln = blocks.classify(mu, nu, 0.0, 1e-1, 0)
    assert nre == 0 and np.array_equal(Ws[0], W)
    ref_u, ref_d = ifherk.step(u0, dt, dx, re, "A", soln_mask=blocks.cell_mask(soln, nb, u0.shape[1:]),
                               supp_mask=blocks.cell_mask(supp, nb, u0.shape[1:]))
    assert np.array_equal(u, ref_u) and np.array_equal(d, ref_d)


def test_run_adaptive_reinitialises_from_the_new_support_when_the_domain_changes():
    """A compact vortex blob in the central blocks: its support domain (W > 0) grows after the first
    step, as the integrating factor carries vorticity into the neighbouring blocks.  The second step
    must re-initialise u from the vorticity on the NEW support (Eq. vel_refresh) before stepping; the
    count of re-initialisations equals the number of changes of the classified masks; the edge flags
    say whether D_xsoln reached the outer block layer."""
    from oracle import blocks

    u0, dx = _compact_velocity()
    shape = u0.shape[1:]
    dt, re, nb, n_buf, es, eo = 0.2, 100.0, 3, 1, 0.0, 1e-1
    u, d, nre, Ws, edge = refresh.run_adaptive(u0, 3, dt, dx, re, "A", n_buf, nb, es, eo, 0)
    masks = [((W > es).astype(np.uint8), (W > eo).astype(np.uint8)) for W in Ws]
    changes = sum(1 for k in range(1, 3) if not (np.array_equal(masks[k][0], masks[k - 1][0])
                                                  and np.array_equal(masks[k][1], masks[k - 1][1])))
    assert nre == changes >= 1
    assert not np.array_equal(masks[1][0], masks[0][0])  # the support grew after the first step
    for W, e in zip(Ws, edge):
        sol = W > eo
        assert e == bool(sol[0].any() or sol[-1].any() or sol[:, 0].any() or sol[:, -1].any()
                         or sol[:, :, 0].any() or sol[:, :, -1].any())
    # the two steps written out: step on the first masks, re-initialise from the new support, step
    cm = [(blocks.cell_mask(s, nb, shape), blocks.cell_mask(o, nb, shape)) for s, o in masks]
    v1, _ = ifherk.step(u0, dt, dx, re, "A", soln_mask=cm[0][1], supp_mask=cm[0][0])
    new = ifherk.vor2vel(cm[1][0] * stencils.curl(v1, dx), dx)
    old = ifherk.vor2vel(cm[0][0] * stencils.curl(v1, dx), dx)
    assert np.abs(new - old).max() > 1e-6 * np.abs(new).max()  # the choice of support matters here
    v2, d2 = ifherk.step(new, dt, dx, re, "A", soln_mask=cm[1][1], supp_mask=cm[1][0])
    u2, dd2, nre2, _, _ = refresh.run_adaptive(u0, 2, dt, dx, re, "A", n_buf, nb, es, eo, 0)
    assert nre2 == 1 and np.array_equal(u2, v2) and np.array_equal(dd2, d2)


def test_run_active_on_the_whole_grid_is_the_adaptive_run():
    """With an expansion of as many blocks as the grid holds, D_xsoln's bounding box is the whole grid at
    every step, and with eps_soln <= eps_supp (so that D_supp lies in D_soln) the active-box run is the
    adaptive run of the same domains, bit for bit."""
    u0, dx = _compact_velocity(n=16, lo=6, hi=10)
    dt, re, nb, n_buf = 0.2, 100.0, 4, 1
    ua, da, nra, nrg, boxes = refresh.run_active(u0, 3, dt, dx, re, "A", n_buf, nb, 1e-3, 1e-4, 4)
    ub, db, nrb, _, _ = refresh.run_adaptive(u0, 3, dt, dx, re, "A", n_buf, nb, 1e-3, 1e-4, 4)
    assert nrg == 0 and all(b == ((0, 0, 0), (4, 4, 4)) for b in boxes)
    assert nra == nrb and np.array_equal(ua, ub) and np.array_equal(da, db)


def _blob_at(n, corner, width, dx, seed):
    rng = np.random.default_rng(seed)
    a = np.zeros((3, n, n, n))
    sl = tuple(slice(c, c + width) for c in corner)
    a[(slice(None),) + sl] = rng.standard_normal((3, width, width, width))
    u = stencils.curl_bar(a, dx)
    return u * (0.5 / np.abs(u).max())


def test_run_active_box_follows_the_flow_and_is_translation_covariant():
    """A compact vortex blob far from the grid faces: the box shrinks to the blob's expanded domain at the
    first step and grows as the integrating factor spreads the vorticity (re-initialisations with box
    changes); the same blob one block further along every axis gives the same fields one block further
    (the LGF solution and the block logic are translation invariant), and the fields vanish outside the
    final box."""
    n, nb, dx, dt, re, n_buf = 40, 4, 0.3, 0.2, 100.0, 1
    args = (3, dt, dx, re, "A", n_buf, nb, 1e-8, 1e-8, 1)
    ua, da, nra, nga, ba = refresh.run_active(_blob_at(n, (16, 16, 16), 3, dx, 4), *args)
    ub, db, nrb, ngb, bb = refresh.run_active(_blob_at(n, (20, 20, 20), 3, dx, 4), *args)
    assert nra == nrb >= 1 and nga == ngb >= 1
    assert ba[0] != ((0, 0, 0), (10, 10, 10))  # the first step already works on a smaller box
    vol = [np.prod([h - l for l, h in zip(*b)]) for b in ba]
    assert vol[-1] > vol[0]  # the box grew with the support
    assert [tuple(tuple(v + 1 for v in c) for c in b) for b in ba] == bb
    assert np.array_equal(ub[:, 4:, 4:, 4:], ua[:, :-4, :-4, :-4]) and np.array_equal(db[4:, 4:, 4:], da[:-4, :-4, :-4])
    lo, hi = ba[-1]
    inside = np.zeros((n, n, n), dtype=bool)
    inside[lo[0] * nb:hi[0] * nb, lo[1] * nb:hi[1] * nb, lo[2] * nb:hi[2] * nb] = True
    assert not ua[:, ~inside].any() and not da[~inside].any() and np.abs(ua[:, inside]).max() > 0

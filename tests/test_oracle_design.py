"""Pins of the design-space oracle (oracle/design.py) against what the
mathematics fixes: group structure and Burnside orbit counts for the symmetry
projection (Sec. 6.1), closed forms of the trigonometric initialization and its
sigmoid projection (Sec. 6.2), special cases and a brute-force loop for the
sensitivity filter (Sec. 5.3), finite differences and textbook isotropic values
for the objectives (Eq. bulk-obj, shear-obj, poisson-relx, poisson-new), and
hand-made histories for the stopping rule (Sec. 6 parameters)."""
import itertools
import math

import numpy as np
import pytest

from oracle import design as D
from oracle import hmgref as O


# ---------------------------------------------------------------- symmetry
def _compose(g, h, n=5):
    """Signed permutation of applying h then g, read off its action on cells."""
    def act(s, c):
        perm, flips = s
        return tuple((n - 1 - c[perm[a]]) if flips[a] else c[perm[a]] for a in range(3))
    return {c: act(g, act(h, c)) for c in itertools.product(range(n), repeat=3)}


@pytest.mark.parametrize("kind,size", [("reflect3", 8), ("reflect6", 48), ("rotate3", 24)])
def test_groups_are_closed_with_known_orders(kind, size):
    G = D.symmetry_group(kind)
    assert len(G) == size
    n = 5
    actions = [_compose(g, ((0, 1, 2), (0, 0, 0)), n) for g in G]
    keyset = {tuple(sorted(a.items())) for a in actions}
    assert len(keyset) == size  # distinct actions
    for g in G:
        for h in G:
            comp = tuple(sorted(_compose(g, h, n).items()))
            assert comp in keyset


def test_subgroups():
    as_set = lambda k: set(D.symmetry_group(k))  # noqa: E731
    assert as_set("reflect3") <= as_set("reflect6")
    assert as_set("rotate3") <= as_set("reflect6")
    # the three mirror planes are not rotations
    assert ((0, 1, 2), (1, 0, 0)) not in as_set("rotate3")


def _bfs_orbit_average(x, n, gens):
    """Independent orbit averaging: orbits by breadth-first closure under the
    generators acting on cells, then the plain mean on each orbit."""
    a = np.asarray(x).reshape(n, n, n)
    out = np.empty_like(a)
    seen = set()
    for c in itertools.product(range(n), repeat=3):
        if c in seen:
            continue
        orbit, stack = {c}, [c]
        while stack:
            u = stack.pop()
            for g in gens:
                v = g(u)
                if v not in orbit:
                    orbit.add(v)
                    stack.append(v)
        seen |= orbit
        m = np.mean([a[z, y, xx] for (xx, y, z) in orbit])
        for (xx, y, z) in orbit:
            out[z, y, xx] = m
    return out.ravel()


def _gens(kind, n):
    fx = lambda c: (n - 1 - c[0], c[1], c[2])  # noqa: E731
    fy = lambda c: (c[0], n - 1 - c[1], c[2])  # noqa: E731
    fz = lambda c: (c[0], c[1], n - 1 - c[2])  # noqa: E731
    sxy = lambda c: (c[1], c[0], c[2])  # noqa: E731  (mirror x = y)
    syz = lambda c: (c[0], c[2], c[1])  # noqa: E731
    szx = lambda c: (c[2], c[1], c[0])  # noqa: E731
    # quarter turns about the axes through the centre
    rx = lambda c: (c[0], n - 1 - c[2], c[1])  # noqa: E731
    ry = lambda c: (c[2], c[1], n - 1 - c[0])  # noqa: E731
    rz = lambda c: (n - 1 - c[1], c[0], c[2])  # noqa: E731
    return {"reflect3": [fx, fy, fz], "reflect6": [fx, fy, fz, sxy, syz, szx],
            "rotate3": [rx, ry, rz]}[kind]


@pytest.mark.parametrize("kind", D.SYMMETRIES)
@pytest.mark.parametrize("n", [4, 5])
def test_symmetrize_equals_orbit_means(kind, n):
    x = np.random.default_rng(3).random(n ** 3)
    got = D.symmetrize(x, (n, n, n), kind)
    ref = _bfs_orbit_average(x, n, _gens(kind, n))
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("kind", D.SYMMETRIES)
@pytest.mark.parametrize("n", [4, 6])
def test_orbit_counts(kind, n):
    x = np.random.default_rng(4).random(n ** 3)
    y = D.symmetrize(x, (n, n, n), kind)
    distinct = len(np.unique(np.round(y, 12)))
    assert distinct == D.orbit_count(n, kind)
    m = n // 2
    if kind == "reflect3":
        assert distinct == m ** 3
    if kind == "reflect6":
        assert distinct == m * (m + 1) * (m + 2) // 6


@pytest.mark.parametrize("kind", D.SYMMETRIES)
def test_symmetrize_projection_properties(kind):
    n = 6
    x = np.random.default_rng(5).random(n ** 3)
    y = D.symmetrize(x, (n, n, n), kind)
    assert abs(y.mean() - x.mean()) < 1e-14
    assert np.abs(D.symmetrize(y, (n, n, n), kind) - y).max() < 1e-14
    a = y.reshape(n, n, n)
    for g in _gens(kind, n):
        for c in itertools.product(range(n), repeat=3):
            d = g(c)
            assert a[c[2], c[1], c[0]] == pytest.approx(a[d[2], d[1], d[0]], abs=1e-14)


def test_reflect3_on_a_box():
    shape = (6, 4, 8)
    x = np.random.default_rng(6).random(np.prod(shape))
    y = D.symmetrize(x, shape, "reflect3").reshape(8, 4, 6)
    assert np.abs(y - y[:, :, ::-1]).max() < 1e-15
    assert np.abs(y - y[:, ::-1, :]).max() < 1e-15
    assert np.abs(y - y[::-1, :, :]).max() < 1e-15
    with pytest.raises(ValueError):
        D.symmetrize(x, shape, "reflect6")


# ---------------------------------------------------------------- initialization
def test_quaternion_rotation():
    R = D.quaternion_rotation([0.3, -0.5, 0.7, 0.1])
    assert np.abs(R @ R.T - np.eye(3)).max() < 1e-14
    assert abs(np.linalg.det(R) - 1) < 1e-14
    assert np.abs(D.quaternion_rotation([2.0, 0, 0, 0]) - np.eye(3)).max() < 1e-15
    # half turn about z: (w, x, y, z) = (0, 0, 0, 1)
    assert np.abs(D.quaternion_rotation([0, 0, 0, 1]) - np.diag([-1, -1, 1])).max() < 1e-15


def test_trig_basis_identity_rotation():
    shape = (4, 6, 8)
    Q = D.trig_basis(shape, 2, [1, 0, 0, 0])
    assert Q.shape == (D.trig_basis_count(2), 4 * 6 * 8)
    assert D.trig_basis_count(2) == 12 + 78
    e = 1 + 4 * (2 + 6 * 3)  # element (1, 2, 3)
    xs = ((1 + 0.5) / 4 - 0.5, (2 + 0.5) / 6 - 0.5, (3 + 0.5) / 8 - 0.5)
    T = []
    for i in range(3):
        for k in (1, 2):
            T += [math.cos(2 * math.pi * k * xs[i]), math.sin(2 * math.pi * k * xs[i])]
    assert np.abs(Q[:12, e] - T).max() < 1e-14
    assert Q[12, e] == pytest.approx(T[0] * T[0], abs=1e-14)
    assert Q[13, e] == pytest.approx(T[0] * T[1], abs=1e-14)
    assert Q[-1, e] == pytest.approx(T[11] * T[11], abs=1e-14)


def test_sigmoid_projection_meets_volume_and_bounds():
    y = np.random.default_rng(7).normal(size=5000)
    for V in (0.1, 0.3, 0.7):
        rho, mu = D.sigmoid_projection(y, V)
        vh = min(1.5 * V, 1.0)
        assert abs(rho.mean() - V) < 1e-12
        assert rho.min() >= 1e-3 and rho.max() <= 1e-3 + vh
        assert np.abs(rho - (1e-3 + vh / (1 + np.exp(-15 * (y - mu))))).max() < 1e-15


def test_trig_init_volume():
    nb = D.trig_basis_count(1)
    w = np.linspace(-1, 1, nb)
    rho, _ = D.trig_init((8, 8, 8), 1, [0.2, 0.4, -0.1, 0.9], w, 0.3)
    assert abs(rho.mean() - 0.3) < 1e-12


# ---------------------------------------------------------------- sensitivity filter
def test_filter_sensitivity_special_cases():
    shape = (6, 5, 4)
    n = np.prod(shape)
    rng = np.random.default_rng(8)
    g = rng.normal(size=n)
    # uniform density: the plain (normalized) cone filter of g
    x = np.full(n, 0.4)
    assert np.abs(D.filter_sensitivity(x, g, shape) - O.density_filter(g, shape, 2.0)).max() < 1e-14
    # g = c / x: x g is constant, so the result is c / max(floor, x)
    x = rng.uniform(1e-4, 1.0, size=n)
    got = D.filter_sensitivity(x, 2.5 / x, shape)
    assert np.abs(got - 2.5 / np.maximum(1e-3, x)).max() < 1e-12 * np.abs(got).max()


def test_filter_sensitivity_brute_force():
    shape = (4, 5, 3)
    nx, ny, nz = shape
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, size=nx * ny * nz)
    x[3] = 1e-5
    g = rng.normal(size=x.size)
    ref = np.zeros_like(x)
    for z, y, xx in itertools.product(range(nz), range(ny), range(nx)):
        num = den = 0.0
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            w = max(0.0, 2.0 - math.sqrt(dx * dx + dy * dy + dz * dz))
            f = (xx + dx) % nx + nx * (((y + dy) % ny) + ny * ((z + dz) % nz))
            num += w * x[f] * g[f]
            den += w
        e = xx + nx * (y + ny * z)
        ref[e] = num / (max(1e-3, x[e]) * den)
    assert np.abs(D.filter_sensitivity(x, g, shape) - ref).max() < 1e-13


# ---------------------------------------------------------------- objectives
@pytest.mark.parametrize("kind", D.OBJECTIVES)
def test_objective_gradients_by_finite_differences(kind):
    rng = np.random.default_rng(10)
    A = rng.normal(size=(6, 6))
    C = A @ A.T + 6 * np.eye(6)
    _, W = D.objective(kind, C, iteration=3)
    h = 1e-6
    for i in range(6):
        for j in range(6):
            Cp, Cm = C.copy(), C.copy()
            Cp[i, j] += h
            Cm[i, j] -= h
            fd = (D.objective(kind, Cp, iteration=3)[0] - D.objective(kind, Cm, iteration=3)[0]) / (2 * h)
            assert abs(fd - W[i, j]) < 1e-7, (i, j, fd, W[i, j])


def test_objectives_on_the_isotropic_base_tensor():
    E, nu = 1.0, 0.3
    lam, mu = O.lame(E, nu)
    Dm = O.constitutive_matrix(E, nu)
    assert D.objective("bulk", Dm)[0] == pytest.approx(-(lam + 2 * mu / 3), abs=1e-15)
    assert D.objective("shear", Dm)[0] == pytest.approx(-mu, abs=1e-15)
    assert D.objective("poisson_relaxed", Dm, iteration=0)[0] == pytest.approx(-6 * mu, abs=1e-14)
    assert D.objective("poisson_relaxed", Dm, iteration=2, beta=0.5)[0] == pytest.approx(
        3 * lam - 0.25 * 3 * (lam + 2 * mu), abs=1e-14)
    want = math.log(1 + 0.6 * nu / (1 - nu)) - math.sqrt(3 * (lam + 2 * mu))
    assert D.objective("poisson_log", Dm)[0] == pytest.approx(want, abs=1e-14)


# ---------------------------------------------------------------- stopping rule
def test_stopping_rule():
    assert not D.should_stop([1.0, 0.5, 0.4])
    assert not D.should_stop([1.0, 1.0001, 1.0002])          # only two changes
    assert D.should_stop([1.0, 1.0001, 1.0002, 1.0003])      # three below 5e-4
    assert not D.should_stop([1.0, 2.0, 2.0001, 2.0002])     # a large change 3 back
    assert not D.should_stop([1.0, 1.0001, 1.001, 1.0011])   # one change of ~9e-4
    assert D.should_stop(list(range(1, 301)))                # 300 iterations
    assert not D.should_stop([-2.0, -2.0004, -2.0008, -2.0025])
    assert D.should_stop([-2.0, -2.0004, -2.0008, -2.0012])

"""Pins of the edge-edge contact oracle (oracle/contact.py): the segment distance against a
brute-force minimum and closed forms, its derivatives against the envelope theorem and
central differences, the pair list against a double loop with the exclusion rule written
out, and friction (Eq. 12-13) in a configuration where the slip velocity is known."""
import math

import numpy as np
import pytest
import torch
from scipy.optimize import minimize

from oracle import contact as K
from oracle import der

DT = torch.float64


def t(*v):
    return torch.tensor(v, dtype=DT)


def brute_distance(a, b, c, d):
    """min over a 201 x 201 grid of (s, t), refined by a bounded quasi-Newton minimiser."""
    a, b, c, d = (np.asarray(v, dtype=float) for v in (a, b, c, d))
    g = np.linspace(0.0, 1.0, 201)
    P = a[None, :] + g[:, None] * (b - a)[None, :]
    Q = c[None, :] + g[:, None] * (d - c)[None, :]
    D2 = ((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1)
    i, j = np.unravel_index(np.argmin(D2), D2.shape)
    f = lambda z: float(((a + z[0] * (b - a) - c - z[1] * (d - c)) ** 2).sum())
    r = minimize(f, [g[i], g[j]], bounds=[(0, 1), (0, 1)], method="L-BFGS-B",
                 options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 500})
    return math.sqrt(min(r.fun, D2[i, j]))


def random_pairs(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        a = rng.normal(size=3)
        u = rng.normal(size=3)
        c = a + rng.normal(size=3) * rng.choice([0.1, 1.0])
        v = rng.normal(size=3)
        if k % 5 == 0:
            v = u * rng.uniform(0.3, 2.0) + 1e-3 * rng.normal(size=3)    # nearly parallel
        out.append((a, a + u, c, c + v))
    return out


def test_distance_against_brute_force_minimum():
    worst = 0.0
    for a, b, c, d in random_pairs(120, 1):
        D, s, tt = K.segment_distance(*(torch.tensor(v, dtype=DT) for v in (a, b, c, d)))
        ref = brute_distance(a, b, c, d)
        worst = max(worst, abs(float(D) - ref))
        # the reported parameters attain the distance
        P = a + float(s) * (b - a)
        Q = c + float(tt) * (d - c)
        assert abs(np.linalg.norm(P - Q) - float(D)) < 1e-12
        assert -1e-15 <= float(s) <= 1 + 1e-15 and -1e-15 <= float(tt) <= 1 + 1e-15
    assert worst < 1e-9


@pytest.mark.parametrize("case,expected", [
    # perpendicular skew segments crossing at their midpoints, 0.3 apart
    ((t(-1, 0, 0), t(1, 0, 0), t(0, -1, 0.3), t(0, 1, 0.3)), (0.3, 0.5, 0.5)),
    # parallel segments, overlapping in projection, 0.2 apart (any overlapping point is closest)
    ((t(0, 0, 0), t(2, 0, 0), t(1, 0.2, 0), t(3, 0.2, 0)), (0.2, None, None)),
    # collinear segments one apart: end point to end point
    ((t(0, 0, 0), t(1, 0, 0), t(2, 0, 0), t(3, 0, 0)), (1.0, 1.0, 0.0)),
    # an end point over the other segment's interior
    ((t(0, 0, 0), t(1, 0, 0), t(0.5, 0.2, 0), t(0.5, 1, 0)), (0.2, 0.5, 0.0)),
    # skew lines whose closest points lie outside both segments: end point b to end of (c, d)
    ((t(0, 0, 0), t(1, 0, 0), t(2, -1, 1), t(2, 1, 1)), (math.sqrt(2.0), 1.0, 0.5)),
])
def test_distance_closed_forms(case, expected):
    D, s, tt = K.segment_distance(*case)
    assert abs(float(D) - expected[0]) < 1e-14
    if expected[1] is not None:
        assert abs(float(s) - expected[1]) < 1e-14 and abs(float(tt) - expected[2]) < 1e-14


def test_distance_symmetries_and_rigid_motion():
    rng = np.random.Generator(np.random.PCG64(3))
    R = torch.tensor(np.linalg.qr(rng.normal(size=(3, 3)))[0], dtype=DT)
    shift = torch.tensor(rng.normal(size=3), dtype=DT)
    for a, b, c, d in random_pairs(40, 2):
        a, b, c, d = (torch.tensor(v, dtype=DT) for v in (a, b, c, d))
        D = float(K.segment_distance(a, b, c, d)[0])
        for perm in ((c, d, a, b), (b, a, c, d), (a, b, d, c), (d, c, b, a)):
            assert abs(float(K.segment_distance(*perm)[0]) - D) < 1e-13
        moved = [R @ v + shift for v in (a, b, c, d)]
        assert abs(float(K.segment_distance(*moved)[0]) - D) < 1e-12


def stable_cases(n, seed):
    """Random pairs with a positive distance whose closest-point pattern (interior or clamped
    at 0 or 1, per parameter) does not change within 1e-4 of the coordinates, so central
    differences stay on one smooth branch."""
    out = []
    for a, b, c, d in random_pairs(n, seed):
        x = torch.tensor(np.concatenate([a, b, c, d]), dtype=DT)

        def pattern(xx):
            _, s, tt = K.segment_distance(xx[0:3], xx[3:6], xx[6:9], xx[9:12])
            return tuple(0 if float(p) <= 0 else (2 if float(p) >= 1 else 1) for p in (s, tt))
        p0 = pattern(x)
        ok = float(K.distance_of(x)) > 1e-3
        for k in range(12):
            for sgn in (-1, 1):
                e = torch.zeros(12, dtype=DT)
                e[k] = sgn * 1e-4
                ok = ok and pattern(x + e) == p0
        if ok:
            out.append(x)
    return out


def test_gradient_is_the_envelope_closed_form_and_matches_differences():
    cases = stable_cases(80, 4)
    assert len(cases) > 40
    for x in cases:
        g = K.distance_gradient(x)
        D, s, tt = K.segment_distance(x[0:3], x[3:6], x[6:9], x[9:12])
        P = x[0:3] + s * (x[3:6] - x[0:3])
        Q = x[6:9] + tt * (x[9:12] - x[6:9])
        n = (P - Q) / D
        closed = torch.cat([(1 - s) * n, s * n, -(1 - tt) * n, -tt * n])
        assert torch.allclose(g, closed, rtol=0, atol=1e-13)
        h = 1e-6
        fd = torch.stack([(K.distance_of(x + h * e) - K.distance_of(x - h * e)) / (2 * h)
                          for e in torch.eye(12, dtype=DT)])
        assert torch.allclose(g, fd, rtol=0, atol=1e-8)


def test_hessian_matches_differences_of_the_gradient():
    for x in stable_cases(60, 5)[:30]:
        H = K.distance_hessian(x)
        assert torch.allclose(H, H.T, atol=1e-12)
        h = 1e-6
        fd = torch.stack([(K.distance_gradient(x + h * e) - K.distance_gradient(x - h * e)) / (2 * h)
                          for e in torch.eye(12, dtype=DT)], 1)
        scale = float(H.abs().max())
        assert float((H - fd).abs().max()) < 1e-6 * max(scale, 1.0)


def test_pair_energy_terms_match_differences():
    C, delta, kc = 0.02, 5e-4, 3.0
    # distances across the soft band and the quadratic branch
    for z in (C - 3 * delta, C - 0.5 * delta, C + 0.3 * delta):
        x = torch.cat([t(-0.1, 0.0, 0.0), t(0.1, 0.01, 0.0), t(0.02, -0.1, z), t(-0.01, 0.1, z)])
        e, g, H = K.pair_terms(x, C, delta, kc)
        h = 1e-8
        fd = torch.stack([(K.pair_energy(x + h * ee, C, delta, kc) - K.pair_energy(x - h * ee, C, delta, kc)) / (2 * h)
                          for ee in torch.eye(12, dtype=DT)])
        assert float((g - fd).abs().max()) < 1e-6 * float(g.abs().max())
        fdH = torch.stack([(K.pair_terms(x + h * ee, C, delta, kc)[1] - K.pair_terms(x - h * ee, C, delta, kc)[1]) / (2 * h)
                           for ee in torch.eye(12, dtype=DT)], 1)
        assert float((H - fdH).abs().max()) < 1e-5 * float(H.abs().max())
        # translation invariance: the forces on the four nodes sum to zero
        assert float(g.view(4, 3).sum(0).abs().max()) < 1e-12 * float(g.abs().max())
    # out of reach: nothing
    x = torch.cat([t(-0.1, 0.0, 0.0), t(0.1, 0.0, 0.0), t(0.0, -0.1, C + 2 * delta), t(0.0, 0.1, C + 2 * delta)])
    e, g, H = K.pair_terms(x, C, delta, kc)
    assert float(e) == 0.0 and float(g.abs().max()) == 0.0


def helix(n, radius, pitch, turns):
    s = np.linspace(0.0, 2 * np.pi * turns, n)
    return np.stack([radius * np.cos(s), radius * np.sin(s), pitch * s / (2 * np.pi)], 1)


def test_pair_list_of_a_tight_helix_and_two_crossing_rods():
    h, delta = 0.004, 5e-4
    # a helix whose turns are 7 mm apart: closer than 2h + delta = 8.5 mm
    x0 = helix(81, 0.02, 0.007, 4.0)
    # two straight rods crossing under the helix, 2h - delta/2 apart at their crossing
    z = -0.05
    r1 = np.stack([np.linspace(-0.1, 0.1, 11), np.zeros(11), np.full(11, z)], 1) + [0.01, 0.0, 0.0]
    r2 = np.stack([np.zeros(11), np.linspace(-0.1, 0.1, 11), np.full(11, z + 2 * h - delta / 2)], 1) + [0.0, 0.01, 0.0]
    es, n = K.EdgeSet.from_rods([(x0, h), (r1, h), (r2, h)])
    x = torch.tensor(np.concatenate([x0, r1, r2]), dtype=DT)
    pairs = K.contact_pairs(es, x, delta)
    got = {(i, j) for (i, j, *_) in pairs}
    # the exclusion rule and the reach written out over every pair
    E = es.edges.shape[0]
    want = set()
    for i in range(E):
        for j in range(i + 1, E):
            same = int(es.rod[i]) == int(es.rod[j])
            if same:
                lo, hi = sorted((int(es.pos[i]), int(es.pos[j])))
                idx = [k for k in range(E) if int(es.rod[k]) == int(es.rod[i]) and lo < int(es.pos[k]) < hi]
                if sum(float(es.ebar[k]) for k in idx) < 2 * h + delta:
                    continue
            a, b = es.edges[i].tolist()
            c, d = es.edges[j].tolist()
            if brute_distance(x[a], x[b], x[c], x[d]) < 2 * h + delta:
                want.add((i, j))
    assert got == want
    helix_pairs = [(i, j) for (i, j) in got if int(es.rod[i]) == 0 and int(es.rod[j]) == 0]
    cross = [(i, j) for (i, j) in got if int(es.rod[i]) != int(es.rod[j])]
    # consecutive turns touch (20 edges per turn), the crossing rods touch once, at their
    # middle edges, and nothing touches across the gap between the helix and the rods
    assert len(helix_pairs) > 40
    assert all(17 <= abs(int(es.pos[j]) - int(es.pos[i])) <= 23 for (i, j) in helix_pairs)
    assert len(cross) == 1
    i, j = cross[0]
    assert int(es.rod[i]) == 1 and int(es.rod[j]) == 2 and int(es.pos[i]) == 4 and int(es.pos[j]) == 4
    # a straight rod alone touches nothing
    es1, _ = K.EdgeSet.from_rods([(r1, h)])
    assert K.contact_pairs(es1, torch.tensor(r1, dtype=DT), delta) == []


def test_contact_force_is_minus_the_energy_gradient_along_the_normal():
    C, delta, kc = 0.01, 5e-4, 2.0
    D0 = C - 0.4 * delta
    x = np.array([[-0.1, 0, 0], [0.1, 0, 0], [0, -0.1, D0], [0, 0.1, D0]], dtype=float)
    es = K.EdgeSet([(0, 1), (2, 3)], [0, 1], [0, 0], [C / 2, C / 2], [0.2, 0.2])
    pairs = K.contact_pairs(es, torch.tensor(x, dtype=DT), delta)
    assert len(pairs) == 1
    F = K.contact_force(es, x, pairs, delta, kc)
    # Eq. 10 in the soft band: E = (log(1 + exp(z)) / K1)^2, z = K1 (C - D)
    K1 = 15.0 / delta
    z = K1 * (C - D0)
    dEdD = -2.0 * math.log1p(math.exp(z)) / K1 * (math.exp(z) / (1.0 + math.exp(z)))
    f = -kc * dEdD          # along +z on the upper edge (D grows with its height)
    assert np.allclose(F[2:].numpy(), [[0, 0, f / 2], [0, 0, f / 2]], rtol=1e-12, atol=0)
    assert np.allclose(F[:2].numpy(), [[0, 0, -f / 2], [0, 0, -f / 2]], rtol=1e-12, atol=0)


def test_friction_against_eq_12_13_for_a_known_slip():
    C, delta, kc, mu, nu, dt = 0.01, 5e-4, 2.0, 0.5, 1e-3, 1e-3
    D0 = C - 0.5 * delta
    x = np.array([[-0.1, 0, 0], [0.1, 0, 0], [0, -0.1, D0], [0, 0.1, D0]], dtype=float)
    for U in (2e-4, 3e-3, 0.05):          # sticking, transition, sliding
        xn = x.copy()
        xn[2:, 0] -= U * dt               # the upper edge moved +U along x over the step
        es = K.EdgeSet([(0, 1), (2, 3)], [0, 1], [0, 0], [C / 2, C / 2], [0.2, 0.2])
        pairs = K.contact_pairs(es, torch.tensor(x, dtype=DT), delta)
        Ffr = K.friction_force(es, x, xn, dt, pairs, delta, kc, mu, nu).numpy()
        K1, K2 = 15.0 / delta, 15.0 / nu
        zz = K1 * (C - D0)
        fcon = kc * 2.0 * math.log1p(math.exp(zz)) / K1 * (math.exp(zz) / (1.0 + math.exp(zz)))
        gamma = 2.0 / (1.0 + math.exp(-K2 * U)) - 1.0
        f = mu * gamma * fcon             # lower edge dragged along +x, upper edge held back
        assert np.allclose(Ffr[:2], [[f / 2, 0, 0], [f / 2, 0, 0]], rtol=1e-12, atol=1e-300)
        assert np.allclose(Ffr[2:], [[-f / 2, 0, 0], [-f / 2, 0, 0]], rtol=1e-12, atol=1e-300)
        # the normal part of the relative velocity carries no friction
        xn2 = x.copy()
        xn2[2:, 2] -= U * dt
        F2 = K.friction_force(es, x, xn2, dt, pairs, delta, kc, mu, nu).numpy()
        assert np.abs(F2).max() == 0.0


def test_the_floor_profile_is_the_one_of_eq_10():
    """The pair energy reuses the floor's Eq. 10 profile: spot values of its three branches."""
    C, delta = 0.01, 5e-4
    K1 = 15.0 / delta
    for D, ref in ((C - 2 * delta, (2 * delta) ** 2),
                   (C, (math.log(2.0) / K1) ** 2),
                   (C + 0.5 * delta, (math.log1p(math.exp(-0.5 * K1 * delta)) / K1) ** 2),
                   (C + delta, 0.0)):
        assert abs(float(der.contact_energy_profile(torch.tensor(D, dtype=DT), C, delta)) - ref) <= 1e-12 * max(ref, 1e-30)

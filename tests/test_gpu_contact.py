"""Edge-edge contact on the GPU (dm_contact_*) against the oracle (oracle/contact.py).

Tolerances: D is one square root of a float64 sum of products on both sides (1e-12
relative); s and t are compared where they are unique (edges not within 1e-6 of parallel,
1e-9); the gradient follows from D, s, t in closed form (1e-10 of its largest entry); the
Hessian's closed form (implicit differentiation of the closest-point conditions) is compared
with the oracle's automatic Hessian through its candidate branches, 1e-8 of the largest entry
for pairs whose edges are not within 1e-3 of parallel (the closed form divides by
|b - a|^2 |d - c|^2 - ((b - a).(d - c))^2, which amplifies rounding near parallel edges).
The pair lists are integer results and must be equal."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import contact as OC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2311_18126_amd as m
    assert os.path.exists(m.LIB_PATH), "libdmrod.so is not built"
    return m


def say(msg):
    print(msg, flush=True)


def scene_edges(rods):
    es, n = OC.EdgeSet.from_rods(rods)
    x = np.concatenate([r[0] for r in rods])
    return es, x


def unpack(pairs, dst, counts):
    """Per group: list of (i, j) and the matching (D, s, t) rows."""
    P, Dd, c = pairs.cpu().numpy(), dst.cpu().numpy(), counts.cpu().numpy()
    return [(P[g, :c[g]], Dd[g, :c[g]]) for g in range(len(c))]


@pytest.fixture(scope="module")
def tangle(dm):
    import torch
    d = W.contact_tangle(3, seed=11)
    c = dm.Contact.from_rods(d["rods"], d["groups"], d["delta"], 512)
    x = torch.tensor(np.concatenate([r[0] for r in d["rods"]]), device="cuda")
    pairs, dst, counts, total = c.find(x)
    say(f"tangle: {total} pairs over {len(d['groups'])} scenes")
    return d, c, x, pairs, dst, counts


def test_pairs_and_distances_match_the_oracle(dm, tangle):
    import torch
    d, c, x, pairs, dst, counts = tangle
    got = unpack(pairs, dst, counts)
    eoff = 0
    for g, gsize in enumerate(d["groups"]):
        rods = d["rods"][5 * g:5 * g + gsize]
        es, xs = scene_edges(rods)
        ref = OC.contact_pairs(es, torch.tensor(xs), d["delta"])
        P, Ds = got[g]
        gp = [(int(i) - eoff, int(j) - eoff) for i, j in P]
        assert gp == [(i, j) for (i, j, *_) in ref]              # same pairs, same order
        D_ref = np.array([r[2] for r in ref])
        assert np.allclose(Ds[:, 0], D_ref, rtol=1e-12, atol=0)
        # s, t where the closest points are unique
        for k, (i, j, D, s, t) in enumerate(ref):
            a, b = es.edges[i].tolist()
            cc, dd = es.edges[j].tolist()
            u, v = xs[b] - xs[a], xs[dd] - xs[cc]
            if np.linalg.norm(np.cross(u, v)) > 1e-6 * np.linalg.norm(u) * np.linalg.norm(v):
                assert abs(Ds[k, 1] - s) < 1e-9 and abs(Ds[k, 2] - t) < 1e-9
        say(f"scene {g}: {len(ref)} pairs equal")
        eoff += es.edges.shape[0]


def test_energy_gradient_hessian_and_friction_match_the_oracle(dm, tangle):
    import torch
    d, c, x, pairs, dst, counts = tangle
    xp = torch.tensor(d["x_prev"][:x.shape[0]], device="cuda")
    E, G, H, F = c.terms(x, pairs, counts, d["k_c"], x_prev=xp, dt=d["dt"], mu=d["mu"], nu=d["nu"], friction=True)
    E, G, H, F = (a.cpu().numpy() for a in (E, G, H, F))
    P, cnt = pairs.cpu().numpy(), counts.cpu().numpy()
    xs = x.cpu().numpy()
    es_all, _ = OC.EdgeSet.from_rods(d["rods"])
    checked = 0
    for g in range(len(cnt)):
        for k in range(0, cnt[g], 3):            # every third pair of each scene
            i, j = int(P[g, k, 0]), int(P[g, k, 1])
            x12 = torch.tensor(OC.pair_coords(es_all, torch.tensor(xs), i, j).numpy())
            C = es_all.contact_distance(i, j)
            e_ref, g_ref, h_ref = (a.numpy() for a in OC.pair_terms(x12, C, d["delta"], d["k_c"]))
            assert abs(E[g, k] - e_ref) <= 1e-12 * abs(e_ref) + 1e-300
            assert np.abs(G[g, :, k] - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
            a, b = es_all.edges[i].tolist()
            cc, dd = es_all.edges[j].tolist()
            u, v = xs[b] - xs[a], xs[dd] - xs[cc]
            if np.linalg.norm(np.cross(u, v)) > 1e-3 * np.linalg.norm(u) * np.linalg.norm(v):
                Hg = H[g, :, k].reshape(12, 12)
                assert np.abs(Hg - h_ref).max() <= 1e-8 * np.abs(h_ref).max()
            checked += 1
    say(f"{checked} pairs' terms checked")
    # friction: per-node sums of the pair forces against the oracle's, scene 0
    gsz = d["groups"][0]
    es, xs0 = scene_edges(d["rods"][:gsz])
    ref_pairs = OC.contact_pairs(es, torch.tensor(xs0), d["delta"])
    Fref = OC.friction_force(es, xs0, d["x_prev"][:xs0.shape[0]], d["dt"], ref_pairs, d["delta"], d["k_c"], d["mu"],
                             d["nu"]).numpy()
    Fg = np.zeros_like(Fref)
    for k in range(cnt[0]):
        i, j = int(P[0, k, 0]), int(P[0, k, 1])
        nodes = list(es.edges[i].tolist()) + list(es.edges[j].tolist())
        for q, nd in enumerate(nodes):
            Fg[nd] += F[0, 3 * q:3 * q + 3, k]
    assert np.abs(Fg - Fref).max() <= 1e-10 * np.abs(Fref).max()
    assert np.abs(Fref).max() > 0


def lattice(nx, ny, ax, by, h=5e-3, seg=5e-3):
    """Single-edge vertical rods on an nx x ny lattice, spacing ax along x and by along y."""
    rods = []
    for i in range(nx):
        for j in range(ny):
            p = np.array([i * ax, j * by, 0.0])
            rods.append((np.stack([p, p + [0.0, 0.0, seg]]), h))
    return rods


def test_a_full_group_of_parallel_edges(dm):
    """2048 one-edge rods (the largest group) on a 32 x 64 lattice, 9 mm apart along x (within
    C + delta = 10.5 mm) and 15 mm along y: exactly the 31 x 64 x-neighbours touch, at D = 9 mm;
    with 1000 slots the call reports the overflow and the exact count."""
    import torch
    rods = lattice(32, 64, 9e-3, 15e-3)
    c = dm.Contact.from_rods(rods, [len(rods)], 5e-4, 2048)
    x = torch.tensor(np.concatenate([r[0] for r in rods]), device="cuda")
    pairs, dst, counts, total = c.find(x)
    assert total == 31 * 64
    P = pairs[0, :total].cpu().numpy()
    want = sorted((i * 64 + j, (i + 1) * 64 + j) for i in range(31) for j in range(64))
    assert [tuple(p) for p in P] == want
    assert np.allclose(dst[0, :total, 0].cpu().numpy(), 9e-3, rtol=1e-12)
    E, G, H, _ = c.terms(x, pairs, counts, 10.0)
    assert np.isfinite(H.cpu().numpy()).all()
    small = dm.Contact.from_rods(rods, [len(rods)], 5e-4, 1000)
    with pytest.raises(dm.DmError, match="capacity"):
        small.find(x)


def test_empty_small_and_excluded_groups(dm):
    """Groups of 0, 1 and 2 edges, a straight rod (every pair out of reach or excluded) and a
    hairpin whose legs run 9 mm apart (pairs across the legs; the bend's neighbours excluded by
    the rest-arclength rule), against the oracle."""
    import torch
    s = np.linspace(0.0, 0.2, 41)
    straight = np.stack([s, np.zeros_like(s), np.zeros_like(s)], 1)
    # hairpin: two legs along x joined by a half circle of radius 4.5 mm
    th = np.linspace(-np.pi / 2, np.pi / 2, 7)[1:-1]
    leg = np.linspace(0.1, 0.0, 21)
    hp = np.concatenate([np.stack([leg, np.full(21, -4.5e-3), np.zeros(21)], 1),
                         np.stack([-4.5e-3 * np.cos(th), 4.5e-3 * np.sin(th), np.zeros(5)], 1),
                         np.stack([leg[::-1], np.full(21, 4.5e-3), np.zeros(21)], 1)])
    one = np.array([[0.5, 0.5, 0.0], [0.5, 0.5, 0.01]])
    two = [np.array([[0.7, 0.0, 0.0], [0.7, 0.01, 0.0]]), np.array([[0.705, 0.005, -0.005], [0.705, 0.005, 0.005]])]
    rods = [(one, 5e-3)] + [(r, 5e-3) for r in two] + [(straight, 5e-3), (hp, 5e-3)]
    groups = [0, 1, 2, 1, 1]
    c = dm.Contact.from_rods(rods, groups, 5e-4, 256)
    x = torch.tensor(np.concatenate([r[0] for r in rods]), device="cuda")
    pairs, dst, counts, total = c.find(x)
    cnt = counts.cpu().numpy()
    assert cnt[0] == 0 and cnt[1] == 0 and cnt[3] == 0
    assert cnt[2] == 1
    es, xs = scene_edges([rods[4]])
    ref = OC.contact_pairs(es, torch.tensor(xs), 5e-4)
    assert len(ref) > 10
    e0 = sum(r[0].shape[0] - 1 for r in rods[:4])
    got = [(int(i) - e0, int(j) - e0) for i, j in pairs[4, :cnt[4]].cpu().numpy()]
    assert got == [(i, j) for (i, j, *_) in ref]


def test_full_size_scenes_sampled(dm):
    """The bench's 4096 scenes: every reported pair is within reach and not excluded (oracle
    distance on a sample of 3000 pairs), a sample of 3000 unreported candidate pairs is out of
    reach, and two whole scenes equal the oracle's pair lists.  Every rod here has 60 nodes
    and radius 5 mm, so edge e is edge e % 59 of rod e // 59; the exclusion rule is written
    out with the rest lengths summed between the two edges."""
    import torch
    d = W.contact_tangle(4096)
    c = dm.Contact.from_rods(d["rods"], d["groups"], d["delta"], 1024)
    x = torch.tensor(np.concatenate([r[0] for r in d["rods"]]), device="cuda")
    pairs, dst, counts, total = c.find(x)
    say(f"4096 scenes: {total} pairs, detection {c.last_find_ms:.3f} ms")
    xs = x.cpu().numpy()
    h, delta = d["rods"][0][1], d["delta"]
    reach = 2 * h + delta
    eb = np.concatenate([np.linalg.norm(np.diff(r[0], axis=0), axis=1) for r in d["rods"]])

    def nodes(e):
        return (e // 59) * 60 + e % 59, (e // 59) * 60 + e % 59 + 1

    def excluded(i, j):
        return i // 59 == j // 59 and eb[i + 1:j].sum() < reach

    def dist(i, j):
        a, b = nodes(i)
        c_, d_ = nodes(j)
        return float(OC.segment_distance(*(torch.tensor(xs[n]) for n in (a, b, c_, d_)))[0])

    P, cnt = pairs.cpu().numpy(), counts.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(9))
    reported = set()
    for g in range(len(cnt)):
        for k in range(cnt[g]):
            reported.add((int(P[g, k, 0]), int(P[g, k, 1])))
    rep = sorted(reported)
    for idx in rng.choice(len(rep), 3000, replace=False):
        i, j = rep[idx]
        assert not excluded(i, j)
        assert dist(i, j) < reach
    per = 5 * 59
    n_out = 0
    while n_out < 3000:
        g = int(rng.integers(len(cnt)))
        i, j = sorted(int(v) for v in g * per + rng.choice(per, 2, replace=False))
        if (i, j) in reported or excluded(i, j):
            continue
        assert dist(i, j) >= reach
        n_out += 1
    for g in (0, len(cnt) - 1):
        es, xg = scene_edges(d["rods"][5 * g:5 * g + 5])
        ref = OC.contact_pairs(es, torch.tensor(xg), d["delta"])
        got = [(int(i) - g * per, int(j) - g * per) for i, j in P[g, :cnt[g]]]
        assert got == [(i, j) for (i, j, *_) in ref]

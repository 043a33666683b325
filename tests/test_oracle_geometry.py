"""Geometry pins: site counts, face structure, tiling conditions, sweep
orders (Sec. "Defining the Kagome block", "Conditions for studying infinite
lattices using BlockBP"; App. "Kagome Block Indexing")."""
import os
from collections import Counter

import pytest

from oracle import geometry as geo

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kagome_block_counts.txt")


def _golden():
    hexes, pars = {}, {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "L":
            pars[int(f[1])] = int(f[2])
        else:
            hexes[int(f[0])] = int(f[1])
    return hexes, pars


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_hex_counts_and_faces(N):
    hexes, _ = _golden()
    P = geo.HexProblem(N)
    assert len(P.net.sites) == hexes[N]
    faces = P.faces[0]
    assert [f["key"] for f in faces] == [("hex", f) for f in range(6)]
    # the same number of legs crosses every face: 2N - 1
    assert [len(f["legs"]) for f in faces] == [2 * N - 1] * 6
    # faces alternate between 2N-1 and N distinct tensors (three-fold symmetry)
    ns = [len({s for s, _ in f["legs"]}) for f in faces]
    assert ns == [2 * N - 1, N] * 3
    # every site has four legs, every leg is a bond or a face leg
    for s in range(len(P.net.sites)):
        for l in range(4):
            assert P.net.link[(s, l)] is not None


@pytest.mark.parametrize("L", [2, 3, 4])
def test_parallelogram_counts(L):
    _, pars = _golden()
    F = geo.FiniteProblem(L, L, L, L)
    assert len(F.blocks) == 1 and len(F.blocks[0]) == pars[L]


@pytest.mark.parametrize("N", [2, 3, 4])
def test_hex_tiling_conditions(N):
    """Condition (i): the translates of the block cover every cell exactly
    once; condition (ii): every leg of face f pairs with a leg of face f+3."""
    P = geo.HexProblem(N)
    cells = set(geo.hex_cells(N))
    R = 3 * N
    for i in range(-R, R + 1):
        for j in range(-R, R + 1):
            hits = 0
            for a in range(-3, 4):
                for b in range(-3, 4):
                    ti = i - a * P.V[2][0] - b * P.V[3][0]
                    tj = j - a * P.V[2][1] - b * P.V[3][1]
                    hits += (ti, tj) in cells
            assert hits == 1
    for f in range(6):
        for sl in P.faces[0][f]["legs"]:
            s2, l2 = P.net.pair[sl]
            assert P.net.link[(s2, l2)] == ("face", (f + 3) % 6)
            assert P.net.pair[(s2, l2)] == sl


def test_finite_patch_counts():
    F = geo.FiniteProblem(4, 4, 2, 2)
    assert len(F.net.sites) == 48
    assert len(F.net.bonds()) == 81
    deg = Counter(sum(F.net.link[(s, l)] is not None for l in range(4)) for s in range(48))
    assert deg == Counter({4: 27, 3: 12, 2: 9})
    inter = [b for b in F.net.bonds() if F.block_of[b[0][0]] != F.block_of[b[1][0]]]
    assert len(inter) == 13
    assert len(F.msg_keys) == 10
    sizes = sorted(len(F.update_target(k)[2]) for k in F.msg_keys)
    assert sizes == [1, 1] + [3] * 8


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_sweeps_are_valid(N):
    """Every direction's sweep keeps in-legs contiguous (asserted inside the
    generator) and ends exactly on the target face, whose legs map onto the
    receiving face in order."""
    P = geo.HexProblem(N)
    for t in range(6):
        steps, final = geo.sweep_schedule(P.net, P.blocks[0], P.faces[0], t)
        assert len(steps) == len(P.net.sites)
        assert final[::-1] == P.faces[0][t]["legs"]
        assert P.update_target(t)[2] == final


def test_sweeps_rotate_with_the_block():
    """120-degree rotation maps U->DL->DR and faces f -> f+2; the sweep
    order of direction f+2 is the rotated order of direction f."""
    P = geo.HexProblem(3)
    net = P.net
    from fractions import Fraction as Fr
    site_at = {st["xy"]: s for s, st in enumerate(net.sites)}

    def rot_site(s):
        # rotate the position by +120 degrees about the centre (1, 1/3) of
        # the up-triangle at cell (0, 0), in exact (X, Y) units
        X, Y = net.sites[s]["xy"]
        u, v = Fr(X) - 1, Fr(Y) - Fr(1, 3)
        X2 = 1 - (u + 3 * v) / 2
        Y2 = Fr(1, 3) + (u - v) / 2
        assert X2.denominator == 1 and Y2.denominator == 1
        s2 = site_at[(int(X2), int(Y2))]
        rot = {"U": "DL", "DL": "DR", "DR": "U"}
        assert net.sites[s2]["kind"] == rot[net.sites[s]["kind"]]
        return s2

    # the map must be a bijection of the block
    img = {rot_site(s) for s in range(len(net.sites))}
    assert len(img) == len(net.sites)
    for t in range(6):
        s1, _ = geo.sweep_schedule(net, P.blocks[0], P.faces[0], t)
        s2, _ = geo.sweep_schedule(net, P.blocks[0], P.faces[0], (t + 2) % 6)
        assert [rot_site(x["site"]) for x in s1] == [x["site"] for x in s2]

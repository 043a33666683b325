"""Kagome geometry, blocks, faces and boundary-MPS sweep orders (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What the thesis fixes and what is read here:

* The kagome lattice is a triangular Bravais lattice whose every site is
  replaced by an up-triangle; three sites per cell, indexed inside a triangle
  in the order Up, Down-Left, Down-Right (Sec. "Defining the Kagome block",
  App. "Kagome Block Indexing").  Cell R = i*a1 + j*a2 with a1 = (1, 0),
  a2 = (1/2, sqrt(3)/2); DL sits at R, DR at R + a1/2, U at R + a2/2.
* Every site has degree four (Sec. "The Kagome Lattice").  A site's virtual
  legs are ordered by bond angle, counter-clockwise from +x.
* Hexagonal block of face length N holds 3N^2-3N+1 up-triangles, i.e.
  N_T = 3(3N^2-3N+1) sites (21 at N=2, 57 at N=3).  It must tile the lattice
  and every edge leaving a face must enter the opposite face together
  (Sec. "Conditions for studying infinite lattices using BlockBP").  The
  tiling used here is the superlattice V1 = N*a1 + (N-1)*a2 and its 60 degree
  rotations; face f of the block is the face crossed by edges going into the
  copy translated by V_f.
* Messages (faces) are ordered counter-clockwise starting from the bottom
  (App. "Kagome Block Indexing").
* The contraction order of each direction is only shown in missing figures
  (Sec. "Contraction Order").  Reading used here: the boundary chain starts as
  all incoming messages except the target's, concatenated counter-clockwise
  starting after the target face; sites are then swallowed greedily, always
  taking, among the sites whose in-legs form a contiguous run of the chain
  (in the site's counter-clockwise leg order), the one farthest from the
  target face (exact integer projection on the direction from the block
  centroid to the target face's leg centroid), ties broken by the transverse
  coordinate.

All geometry is done in exact integer arithmetic: a point is (X, Y) with real
position (X/4, sqrt(3)*Y/4), so dot products are X1*X2 + 3*Y1*Y2 and cross
products are proportional to X1*Y2 - Y1*X2.
"""
from __future__ import annotations

import functools

KINDS = ("U", "DL", "DR")
KIND_INDEX = {k: n for n, k in enumerate(KINDS)}
KIND_XY = {"DL": (0, 0), "DR": (2, 0), "U": (1, 1)}
# bond vector (in X, Y units) for direction n * 60 degrees
BOND_VEC = [(2, 0), (1, 1), (-1, 1), (-2, 0), (-1, -1), (1, -1)]
# kind -> legs in counter-clockwise order: (direction, neighbour kind, cell offset)
NEIGH = {
    "DL": [(0, "DR", (0, 0)), (1, "U", (0, 0)), (3, "DR", (-1, 0)), (4, "U", (0, -1))],
    "DR": [(0, "DL", (1, 0)), (2, "U", (0, 0)), (3, "DL", (0, 0)), (5, "U", (1, -1))],
    "U": [(1, "DL", (0, 1)), (2, "DR", (-1, 1)), (4, "DL", (0, 0)), (5, "DR", (0, 0))],
}


def site_xy(cell, kind):
    i, j = cell
    dx, dy = KIND_XY[kind]
    return (4 * i + 2 * j + dx, 2 * j + dy)


def dot(a, b):
    return a[0] * b[0] + 3 * a[1] * b[1]


def cross(a, b):
    return a[0] * b[1] - a[1] * b[0]


def _half(v):
    # angle measured counter-clockwise from -90 degrees (pointing down)
    x, y = v
    return 0 if (x > 0 or (x == 0 and y < 0)) else 1


def angle_cmp(a, b):
    ha, hb = _half(a), _half(b)
    if ha != hb:
        return -1 if ha < hb else 1
    c = cross(a, b)
    if c != 0:
        return -1 if c > 0 else 1
    la, lb = dot(a, a), dot(b, b)
    return (la > lb) - (la < lb)


class Network:
    """Sites of a kagome PEPS with their legs.

    ``sites[s]`` is a dict with keys ``cell``, ``kind``, ``xy``, ``tensor``
    (index of its ket tensor) and ``dirs`` (bond direction of each leg slot).
    ``link[(s, l)]`` is the other end ``(s2, l2)`` inside the network, or
    ``None`` for a leg that leaves a finite patch (dimension 1), or
    ``("face", f)`` for a leg crossing face f of an infinite block.
    """

    def __init__(self):
        self.sites = []
        self.link = {}
        self.pair = {}   # infinite block: (s, l) -> (s2, l2) periodic image

    def nslots(self, s):
        return len(self.sites[s]["dirs"])

    def leg_point(self, s, l):
        """Twice the midpoint of leg l of site s, in (X, Y) units."""
        x, y = self.sites[s]["xy"]
        bx, by = BOND_VEC[self.sites[s]["dirs"][l]]
        return (2 * x + bx, 2 * y + by)

    def bonds(self):
        """Internal bonds ((s1, l1), (s2, l2)) with s1 < s2, sorted."""
        out = []
        for (s, l), o in sorted(self.link.items()):
            if isinstance(o, tuple) and len(o) == 2 and o[0] != "face" and s < o[0]:
                out.append(((s, l), o))
        return out


def _add_cells(net, cells, tensor_of):
    index = {}
    for c in cells:
        for k in KINDS:
            s = len(net.sites)
            net.sites.append({"cell": c, "kind": k, "xy": site_xy(c, k),
                              "tensor": tensor_of(c, k),
                              "dirs": [d for d, _, _ in NEIGH[k]]})
            index[(c, k)] = s
    return index


# ---------------------------------------------------------------- finite patch
class FiniteProblem:
    """Open kagome patch of Lx x Ly cells cut into parallelogram blocks of
    bLx x bLy cells (the thesis's parallelogram block, Sec. "Parallelogram
    block").  Legs leaving the patch have dimension 1; each is a one-leg
    "outside" face whose message is the trivial vector [1]."""

    kind = "finite"

    def __init__(self, Lx, Ly, bLx=None, bLy=None, block_of_cell=None):
        self.Lx, self.Ly = Lx, Ly
        cells = [(i, j) for j in range(Ly) for i in range(Lx)]
        net = Network()
        idx = _add_cells(net, cells, lambda c, k: 3 * (c[1] * Lx + c[0]) + KIND_INDEX[k])
        for (c, k), s in idx.items():
            for l, (d, k2, off) in enumerate(NEIGH[k]):
                c2 = (c[0] + off[0], c[1] + off[1])
                if (c2, k2) in idx:
                    s2 = idx[(c2, k2)]
                    l2 = [n for n, (dd, _, _) in enumerate(NEIGH[k2]) if dd == (d + 3) % 6][0]
                    net.link[(s, l)] = (s2, l2)
                else:
                    net.link[(s, l)] = None
        self.net = net
        if block_of_cell is None:
            nbx = Lx // bLx
            block_of_cell = lambda c: (c[1] // bLy) * nbx + (c[0] // bLx)
        nb = 1 + max(block_of_cell(c) for c in cells)
        self.blocks = [[] for _ in range(nb)]
        self.block_of = {}
        for s, st in enumerate(net.sites):
            b = block_of_cell(st["cell"])
            self.blocks[b].append(s)
            self.block_of[s] = b
        self.faces = [block_faces(net, self.blocks[b], self._key_fn(b)) for b in range(nb)]
        # directed messages (a -> b), ordered by sender then by the sender's face order
        self.msg_keys = []
        for a in range(nb):
            for f in self.faces[a]:
                if f["key"][0] == "block":
                    self.msg_keys.append((a, f["key"][1]))

    def _key_fn(self, b):
        def key(s, l):
            o = self.net.link[(s, l)]
            if o is None:
                return ("outside", s, l)     # every off-patch leg is its own face
            return ("block", self.block_of[o[0]])
        return key

    def face_index(self, b, key):
        for n, f in enumerate(self.faces[b]):
            if f["key"] == key:
                return n
        raise KeyError(key)

    def incoming_key(self, b, face):
        """Message key feeding face ``face`` of block b (None: trivial)."""
        k = self.faces[b][face]["key"]
        return (k[1], b) if k[0] == "block" else None

    def update_target(self, key):
        """(block, target face index, receiving legs in storage order)."""
        a, b = key
        fa = self.face_index(a, ("block", b))
        fb = self.face_index(b, ("block", a))
        # the receiving block's legs, mapped back to the sender's leg ids
        recv = [self.net.link[sl] for sl in self.faces[b][fb]["legs"]]
        return a, fa, recv


# ------------------------------------------------------------ infinite block
def hex_cells(N):
    """Cells of the hexagonal block of face length N (ordered by row, then i)."""
    R = N - 1
    cells = [(i, j) for j in range(-R, R + 1) for i in range(-R, R + 1)
             if abs(i + j) <= R]
    return cells


def rot60(v):
    i, j = v
    return (-j, i + j)


class HexProblem:
    """Single hexagonal block of the infinite kagome lattice sending messages
    to itself (Alg. BlockBP_singleBlock).  Three unique site tensors, one per
    kind (the 3-site unit cell)."""

    kind = "infinite"

    def __init__(self, N):
        if N < 2:
            raise ValueError("hexagonal block needs face length N >= 2")
        self.N = N
        cells = hex_cells(N)
        cellset = set(cells)
        V = [(N, N - 1)]
        for _ in range(5):
            V.append(rot60(V[-1]))
        # face of each translation: the face normal (270 + 60 f degrees) nearest to V
        # V1 points at angle in (0, 30) degrees -> face 2; rotation by 60 adds one face.
        self.V = [None] * 6
        for k in range(6):
            self.V[(2 + k) % 6] = V[k]
        net = Network()
        idx = _add_cells(net, cells, lambda c, k: KIND_INDEX[k])
        for (c, k), s in idx.items():
            for l, (d, k2, off) in enumerate(NEIGH[k]):
                c2 = (c[0] + off[0], c[1] + off[1])
                l2 = [n for n, (dd, _, _) in enumerate(NEIGH[k2]) if dd == (d + 3) % 6][0]
                if c2 in cellset:
                    net.link[(s, l)] = (idx[(c2, k2)], l2)
                    continue
                hits = [f for f in range(6)
                        if (c2[0] - self.V[f][0], c2[1] - self.V[f][1]) in cellset]
                if len(hits) != 1:
                    raise ValueError("tiling condition violated")
                f = hits[0]
                c3 = (c2[0] - self.V[f][0], c2[1] - self.V[f][1])
                net.link[(s, l)] = ("face", f)
                net.pair[(s, l)] = (idx[(c3, k2)], l2)
        self.net = net
        self.blocks = [list(range(len(net.sites)))]
        self.block_of = {s: 0 for s in range(len(net.sites))}
        faces = block_faces(net, self.blocks[0], lambda s, l: ("hex", net.link[(s, l)][1]))
        byf = {f["key"][1]: f for f in faces}
        if sorted(byf) != list(range(6)):
            raise ValueError("expected six faces")
        # faces must follow each other counter-clockwise in index order
        order = [f["key"][1] for f in faces]
        st = order.index(0)
        if order[st:] + order[:st] != list(range(6)):
            raise ValueError("faces are not in counter-clockwise index order")
        self.faces = [[byf[f] for f in range(6)]]
        for f in range(6):
            for sl in self.faces[0][f]["legs"]:
                s2, l2 = net.pair[sl]
                if net.link[(s2, l2)] != ("face", (f + 3) % 6):
                    raise ValueError("edges of a face must enter the opposite face")
        self.msg_keys = list(range(6))

    def incoming_key(self, b, face):
        return face

    def update_target(self, key):
        """Message computed toward face f is stored on the opposite face."""
        f = key
        recv_face = (f + 3) % 6
        recv = [self.net.pair[sl] for sl in self.faces[0][recv_face]["legs"]]
        return 0, f, recv

    def store_key(self, f):
        return (f + 3) % 6

    def central_bonds(self):
        """The six unique bonds of the unit cell at cell (0, 0): three inside
        the up-triangle and three to the neighbouring cells (Sec. "Modes")."""
        net = self.net
        s_of = {(st["cell"], st["kind"]): s for s, st in enumerate(net.sites)}
        u, dl, dr = (s_of[((0, 0), k)] for k in ("U", "DL", "DR"))
        pairs = [(u, dl), (u, dr), (dl, dr),
                 (dr, s_of[((1, 0), "DL")]),
                 (u, s_of[((0, 1), "DL")]),
                 (u, s_of[((-1, 1), "DR")])]
        return pairs


# --------------------------------------------------------------- block faces
def block_faces(net, sites, key_fn):
    """Boundary legs of a block in counter-clockwise order around the block
    centroid, grouped into faces (maximal cyclic runs with the same key).

    Returns a list of faces ``{"key", "legs"}``, each face's legs in
    counter-clockwise order; faces are ordered by the position of their first
    leg in the counter-clockwise order that starts pointing down."""
    inside = set(sites)
    n = len(sites)
    sx = sum(net.sites[s]["xy"][0] for s in sites)
    sy = sum(net.sites[s]["xy"][1] for s in sites)
    legs = []
    for s in sites:
        for l in range(net.nslots(s)):
            o = net.link[(s, l)]
            if isinstance(o, tuple) and len(o) == 2 and o[0] != "face" and o[0] in inside:
                continue
            px, py = net.leg_point(s, l)
            v = (n * px - 2 * sx, n * py - 2 * sy)
            legs.append((v, (s, l)))
    legs.sort(key=functools.cmp_to_key(lambda a, b: angle_cmp(a[0], b[0])))
    keys = [key_fn(*sl) for _, sl in legs]
    m = len(legs)
    if m == 0:
        return []
    starts = [i for i in range(m) if keys[i] != keys[i - 1]]
    if not starts:
        return [{"key": keys[0], "legs": [sl for _, sl in legs]}]
    faces = []
    for si, st in enumerate(starts):
        en = starts[(si + 1) % len(starts)]
        idxs = [(st + t) % m for t in range((en - st) % m or m)]
        faces.append({"key": keys[st], "legs": [legs[i][1] for i in idxs], "first": st})
    faces.sort(key=lambda f: f["first"])
    seen = set()
    for f in faces:
        if f["key"][0] != "outside":
            if f["key"] in seen:
                raise ValueError("a neighbour touches the block along two faces")
            seen.add(f["key"])
        del f["first"]
    return faces


# ------------------------------------------------------------ sweep schedule
def sweep_schedule(net, sites, faces, target, open_sites=()):
    """Order in which a boundary chain swallows the sites of a block.

    The chain starts as the legs of every face except ``target``, taken
    counter-clockwise starting with the face after ``target``.  A leg of the
    chain is named ("in", s, l) when it enters the unswallowed site s at slot
    l, and ("T", s, l) when it is a leg of swallowed site s crossing the
    target face.  Returns ``(steps, final)`` where each step is a dict with
    ``site``, ``pos`` (chain index of its in-legs), ``in_slots`` and
    ``out_slots`` (both in chain order), ``out_ids``, ``open`` and ``absorb``
    (for a site left with no out-leg: "right"/"left" neighbour that takes
    the remaining bond matrix, else None); ``final``
    is the list of (s, l) target legs in chain order.
    """
    inside = set(sites)
    nf = len(faces)
    chain = []
    for k in range(1, nf):
        for (s, l) in faces[(target + k) % nf]["legs"]:
            chain.append(("in", s, l))
    target_legs = set(faces[target]["legs"])
    n = len(sites)
    sx = sum(net.sites[s]["xy"][0] for s in sites)
    sy = sum(net.sites[s]["xy"][1] for s in sites)
    fx = sum(net.leg_point(s, l)[0] for s, l in faces[target]["legs"])
    fy = sum(net.leg_point(s, l)[1] for s, l in faces[target]["legs"])
    k = len(faces[target]["legs"])
    # direction toward the target face: centroid of its leg points minus block centroid
    d = (n * fx - 2 * k * sx, n * fy - 2 * k * sy)

    def sortkey(s):
        x, y = net.sites[s]["xy"]
        v = (n * 2 * x - 2 * sx, n * 2 * y - 2 * sy)
        return (dot(v, d), cross(v, d))

    remaining = set(sites)
    steps = []
    while remaining:
        best = None
        pos_of = {leg: i for i, leg in enumerate(chain)}
        for s in remaining:
            deg = net.nslots(s)
            ins = [l for l in range(deg) if ("in", s, l) in pos_of]
            if not ins:
                continue
            r = len(ins)
            p0 = min(pos_of[("in", s, l)] for l in ins)
            run = chain[p0:p0 + r]
            if any(leg[0] != "in" or leg[1] != s for leg in run):
                continue
            run_slots = [leg[2] for leg in run]
            st = run_slots[0]
            if any(run_slots[t] != (st + t) % deg for t in range(r)):
                continue
            key = sortkey(s)
            if best is None or key < best[0]:
                best = (key, s, p0, run_slots)
        if best is None:
            raise ValueError("no site can be swallowed with contiguous in-legs")
        _, s, p0, run_slots = best
        deg = net.nslots(s)
        r = len(run_slots)
        st = run_slots[0]
        out_ccw = [(st + r + t) % deg for t in range(deg - r)]
        out_slots = out_ccw[::-1]
        out_ids = []
        for l in out_slots:
            if (s, l) in target_legs:
                out_ids.append(("T", s, l))
            else:
                o = net.link[(s, l)]
                if not (isinstance(o, tuple) and len(o) == 2 and o[0] in inside):
                    raise ValueError("out-leg leaves the block off the target face")
                out_ids.append(("in", o[0], o[1]))
        # a site whose legs are all in leaves a bond matrix that is absorbed
        # into the chain site to its right (or to its left at the chain end)
        absorb = None
        if not out_slots:
            absorb = "right" if p0 + r < len(chain) else "left"
            if len(chain) == r:
                raise ValueError("chain would become empty")
        steps.append({"site": s, "pos": p0, "in_slots": run_slots,
                      "out_slots": out_slots, "out_ids": out_ids,
                      "open": s in open_sites, "absorb": absorb})
        chain[p0:p0 + r] = out_ids
        remaining.discard(s)
    if any(leg[0] != "T" for leg in chain):
        raise ValueError("final chain is not the target face")
    final = [(leg[1], leg[2]) for leg in chain]
    if sorted(final) != sorted(faces[target]["legs"]):
        raise ValueError("final chain misses target legs")
    return steps, final

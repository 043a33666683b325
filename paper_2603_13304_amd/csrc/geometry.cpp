// Kagome geometry and boundary-chain sweep orders (see geometry.hpp).
#include "geometry.hpp"

#include <algorithm>
#include <map>
#include <set>

namespace pn {
namespace {

// bond vector of direction n * 60 degrees, in (X, Y) units
const int kBond[6][2] = {{2, 0}, {1, 1}, {-1, 1}, {-2, 0}, {-1, -1}, {1, -1}};
// per kind: slot -> (direction, neighbour kind, cell offset)
struct Nb { int dir, kind, di, dj; };
const Nb kNeigh[3][4] = {
    /* U  */ {{1, KIND_DL, 0, 1}, {2, KIND_DR, -1, 1}, {4, KIND_DL, 0, 0}, {5, KIND_DR, 0, 0}},
    /* DL */ {{0, KIND_DR, 0, 0}, {1, KIND_U, 0, 0}, {3, KIND_DR, -1, 0}, {4, KIND_U, 0, -1}},
    /* DR */ {{0, KIND_DL, 1, 0}, {2, KIND_U, 0, 0}, {3, KIND_DL, 0, 0}, {5, KIND_U, 1, -1}},
};
const int kKindXY[3][2] = {{1, 1}, {0, 0}, {2, 0}};

int slot_with_dir(int kind, int dir) {
  for (int l = 0; l < 4; ++l)
    if (kNeigh[kind][l].dir == dir) return l;
  return -1;
}

// real dot / cross (up to positive factors) in (X, Y) units
inline int64_t rdot(int64_t ax, int64_t ay, int64_t bx, int64_t by) { return ax * bx + 3 * ay * by; }
inline int64_t rcross(int64_t ax, int64_t ay, int64_t bx, int64_t by) { return ax * by - ay * bx; }

// counter-clockwise order starting from the downward direction
bool angle_less(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  int ha = (ax > 0 || (ax == 0 && ay < 0)) ? 0 : 1;
  int hb = (bx > 0 || (bx == 0 && by < 0)) ? 0 : 1;
  if (ha != hb) return ha < hb;
  int64_t c = rcross(ax, ay, bx, by);
  if (c != 0) return c > 0;
  return rdot(ax, ay, ax, ay) < rdot(bx, by, bx, by);
}

void add_cells(Problem* P, const std::vector<std::pair<int, int>>& cells, bool per_cell_tensor,
               std::map<std::tuple<int, int, int>, int>* index) {
  for (size_t c = 0; c < cells.size(); ++c) {
    for (int k = 0; k < 3; ++k) {
      Site st;
      st.ci = cells[c].first;
      st.cj = cells[c].second;
      st.kind = k;
      st.X = 4 * st.ci + 2 * st.cj + kKindXY[k][0];
      st.Y = 2 * st.cj + kKindXY[k][1];
      st.tensor = per_cell_tensor ? int(3 * c + k) : k;
      st.nslot = 4;
      for (int l = 0; l < 4; ++l) st.dirs[l] = kNeigh[k][l].dir;
      (*index)[{st.ci, st.cj, k}] = int(P->sites.size());
      P->sites.push_back(st);
    }
  }
  P->links.assign(P->sites.size(), {});
}

struct FaceKeyT { int type, key; };

std::string block_faces(const Problem& P, const std::vector<int>& sites,
                        const std::vector<std::array<FaceKeyT, 4>>& keys,
                        std::vector<Face>* faces) {
  std::set<int> inside(sites.begin(), sites.end());
  int64_t n = int64_t(sites.size());
  int64_t sx = 0, sy = 0;
  for (int s : sites) { sx += P.sites[s].X; sy += P.sites[s].Y; }
  struct L { int64_t vx, vy; int s, l; };
  std::vector<L> legs;
  for (int s : sites) {
    for (int l = 0; l < P.sites[s].nslot; ++l) {
      const Link& k = P.links[s][l];
      if (k.type == LINK_SITE && inside.count(k.s2)) continue;
      auto pt = P.leg_point(s, l);
      legs.push_back({n * pt.first - 2 * sx, n * pt.second - 2 * sy, s, l});
    }
  }
  std::stable_sort(legs.begin(), legs.end(), [](const L& a, const L& b) {
    return angle_less(a.vx, a.vy, b.vx, b.vy);
  });
  faces->clear();
  size_t m = legs.size();
  if (m == 0) return "";
  auto key_of = [&](size_t i) { return keys[legs[i].s][legs[i].l]; };
  auto same = [&](size_t i, size_t j) {
    FaceKeyT a = key_of(i), b = key_of(j);
    return a.type == b.type && a.key == b.key;
  };
  std::vector<size_t> starts;
  for (size_t i = 0; i < m; ++i)
    if (!same(i, (i + m - 1) % m)) starts.push_back(i);
  if (starts.empty()) {
    Face f;
    f.keytype = key_of(0).type;
    f.key = key_of(0).key;
    for (auto& x : legs) f.legs.push_back({x.s, x.l});
    faces->push_back(f);
    return "";
  }
  std::vector<std::pair<size_t, Face>> tmp;
  for (size_t k = 0; k < starts.size(); ++k) {
    size_t st = starts[k], en = starts[(k + 1) % starts.size()];
    size_t len = (en + m - st) % m;
    if (len == 0) len = m;
    Face f;
    f.keytype = key_of(st).type;
    f.key = key_of(st).key;
    for (size_t t = 0; t < len; ++t) {
      const L& x = legs[(st + t) % m];
      f.legs.push_back({x.s, x.l});
    }
    tmp.push_back({st, f});
  }
  std::stable_sort(tmp.begin(), tmp.end(),
                   [](const std::pair<size_t, Face>& a, const std::pair<size_t, Face>& b) {
                     return a.first < b.first;
                   });
  std::set<int> seen;
  for (auto& x : tmp) {
    if (x.second.keytype == FACE_BLOCK) {
      if (seen.count(x.second.key)) return "a neighbour touches the block along two faces";
      seen.insert(x.second.key);
    }
    faces->push_back(x.second);
  }
  return "";
}

}  // namespace

int Problem::n_tensors() const {
  int m = 0;
  for (auto& s : sites) m = std::max(m, s.tensor + 1);
  return m;
}

std::pair<int64_t, int64_t> Problem::leg_point(int s, int l) const {
  const Site& st = sites[s];
  return {2 * st.X + kBond[st.dirs[l]][0], 2 * st.Y + kBond[st.dirs[l]][1]};
}

int Problem::face_index(int b, int keytype, int key) const {
  for (size_t n = 0; n < faces[b].size(); ++n)
    if (faces[b][n].keytype == keytype && faces[b][n].key == key) return int(n);
  return -1;
}

void Problem::update_target(int m, int* block, int* face,
                            std::vector<std::pair<int, int>>* recv) const {
  recv->clear();
  if (kind == 0) {
    int a = msg_keys[m].first, b = msg_keys[m].second;
    *block = a;
    *face = face_index(a, FACE_BLOCK, b);
    int fb = face_index(b, FACE_BLOCK, a);
    for (auto& sl : faces[b][fb].legs) {
      const Link& k = links[sl.first][sl.second];
      recv->push_back({k.s2, k.l2});
    }
  } else {
    int f = msg_keys[m].first;
    *block = 0;
    *face = f;
    for (auto& sl : faces[0][(f + 3) % 6].legs) {
      const Link& k = links[sl.first][sl.second];
      recv->push_back({k.s2, k.l2});
    }
  }
}

int Problem::incoming_msg(int b, int f) const {
  const Face& F = faces[b][f];
  if (kind == 1) return F.key;  // hex face g is fed by the message stored in slot g
  if (F.keytype != FACE_BLOCK) return -1;
  for (size_t m = 0; m < msg_keys.size(); ++m)
    if (msg_keys[m].first == F.key && msg_keys[m].second == b) return int(m);
  return -1;
}

const std::vector<std::pair<int, int>>& Problem::stored_legs(int m) const {
  if (kind == 1) return faces[0][m].legs;
  int a = msg_keys[m].first, b = msg_keys[m].second;
  return faces[b][face_index(b, FACE_BLOCK, a)].legs;
}

int Problem::stored_slot_of_update(int m) const { return kind == 1 ? (m + 3) % 6 : m; }

std::vector<std::pair<int, int>> Problem::central_bonds() const {
  std::map<std::tuple<int, int, int>, int> at;
  for (size_t s = 0; s < sites.size(); ++s) at[{sites[s].ci, sites[s].cj, sites[s].kind}] = int(s);
  int u = at[{0, 0, KIND_U}], dl = at[{0, 0, KIND_DL}], dr = at[{0, 0, KIND_DR}];
  return {{u, dl}, {u, dr}, {dl, dr},
          {dr, at[{1, 0, KIND_DL}]}, {u, at[{0, 1, KIND_DL}]}, {u, at[{-1, 1, KIND_DR}]}};
}

std::vector<std::pair<int, int>> Problem::bonds() const {
  std::vector<std::pair<int, int>> out;
  for (size_t s = 0; s < sites.size(); ++s)
    for (int l = 0; l < sites[s].nslot; ++l) {
      const Link& k = links[s][l];
      if (k.type == LINK_SITE && int(s) < k.s2) out.push_back({int(s), k.s2});
    }
  return out;
}

std::string build_finite(Problem* P, int Lx, int Ly, int bLx, int bLy) {
  if (Lx <= 0 || Ly <= 0 || bLx <= 0 || bLy <= 0 || Lx % bLx || Ly % bLy)
    return "patch size must be a positive multiple of the block size";
  *P = Problem();
  P->kind = 0;
  P->Lx = Lx; P->Ly = Ly; P->bLx = bLx; P->bLy = bLy;
  std::vector<std::pair<int, int>> cells;
  for (int j = 0; j < Ly; ++j)
    for (int i = 0; i < Lx; ++i) cells.push_back({i, j});
  std::map<std::tuple<int, int, int>, int> idx;
  add_cells(P, cells, true, &idx);
  for (size_t s = 0; s < P->sites.size(); ++s) {
    const Site& st = P->sites[s];
    for (int l = 0; l < 4; ++l) {
      const Nb& nb = kNeigh[st.kind][l];
      auto it = idx.find({st.ci + nb.di, st.cj + nb.dj, nb.kind});
      Link k;
      if (it != idx.end()) {
        k.type = LINK_SITE;
        k.s2 = it->second;
        k.l2 = slot_with_dir(nb.kind, (nb.dir + 3) % 6);
      }
      P->links[s][l] = k;
    }
  }
  int nbx = Lx / bLx, nby = Ly / bLy;
  P->blocks.assign(nbx * nby, {});
  P->block_of.assign(P->sites.size(), 0);
  for (size_t s = 0; s < P->sites.size(); ++s) {
    int b = (P->sites[s].cj / bLy) * nbx + (P->sites[s].ci / bLx);
    P->blocks[b].push_back(int(s));
    P->block_of[s] = b;
  }
  std::vector<std::array<FaceKeyT, 4>> keys(P->sites.size());
  for (size_t s = 0; s < P->sites.size(); ++s)
    for (int l = 0; l < 4; ++l) {
      const Link& k = P->links[s][l];
      if (k.type == LINK_SITE) keys[s][l] = {FACE_BLOCK, P->block_of[k.s2]};
      else keys[s][l] = {FACE_OUTSIDE, int(s) * 8 + l};  // each off-patch leg is its own face
    }
  P->faces.resize(P->blocks.size());
  for (size_t b = 0; b < P->blocks.size(); ++b) {
    std::string e = block_faces(*P, P->blocks[b], keys, &P->faces[b]);
    if (!e.empty()) return e;
  }
  for (size_t a = 0; a < P->blocks.size(); ++a)
    for (auto& f : P->faces[a])
      if (f.keytype == FACE_BLOCK) P->msg_keys.push_back({int(a), f.key});
  return "";
}

std::string build_hex(Problem* P, int N) {
  if (N < 2) return "hexagonal block needs face length N >= 2";
  *P = Problem();
  P->kind = 1;
  P->N = N;
  int R = N - 1;
  std::vector<std::pair<int, int>> cells;
  for (int j = -R; j <= R; ++j)
    for (int i = -R; i <= R; ++i)
      if (std::abs(i + j) <= R) cells.push_back({i, j});
  std::set<std::pair<int, int>> cellset(cells.begin(), cells.end());
  // V1 = (N, N-1) points between 0 and 30 degrees: face 2; each 60-degree
  // rotation (i, j) -> (-j, i + j) advances one face
  int vi = N, vj = N - 1;
  for (int k = 0; k < 6; ++k) {
    P->V[(2 + k) % 6][0] = vi;
    P->V[(2 + k) % 6][1] = vj;
    int ni = -vj, nj = vi + vj;
    vi = ni; vj = nj;
  }
  std::map<std::tuple<int, int, int>, int> idx;
  add_cells(P, cells, false, &idx);
  for (size_t s = 0; s < P->sites.size(); ++s) {
    const Site& st = P->sites[s];
    for (int l = 0; l < 4; ++l) {
      const Nb& nb = kNeigh[st.kind][l];
      int c2i = st.ci + nb.di, c2j = st.cj + nb.dj;
      int l2 = slot_with_dir(nb.kind, (nb.dir + 3) % 6);
      Link k;
      if (cellset.count({c2i, c2j})) {
        k.type = LINK_SITE;
        k.s2 = idx[{c2i, c2j, nb.kind}];
        k.l2 = l2;
      } else {
        int hit = -1, nhit = 0;
        for (int f = 0; f < 6; ++f)
          if (cellset.count({c2i - P->V[f][0], c2j - P->V[f][1]})) { hit = f; ++nhit; }
        if (nhit != 1) return "tiling condition violated";
        k.type = LINK_FACE;
        k.face = hit;
        k.s2 = idx[{c2i - P->V[hit][0], c2j - P->V[hit][1], nb.kind}];
        k.l2 = l2;
      }
      P->links[s][l] = k;
    }
  }
  P->blocks.assign(1, {});
  P->block_of.assign(P->sites.size(), 0);
  for (size_t s = 0; s < P->sites.size(); ++s) P->blocks[0].push_back(int(s));
  std::vector<std::array<FaceKeyT, 4>> keys(P->sites.size());
  for (size_t s = 0; s < P->sites.size(); ++s)
    for (int l = 0; l < 4; ++l) keys[s][l] = {FACE_HEX, P->links[s][l].face};
  std::vector<Face> faces;
  std::string e = block_faces(*P, P->blocks[0], keys, &faces);
  if (!e.empty()) return e;
  if (faces.size() != 6) return "expected six faces";
  std::vector<Face> byf(6);
  int first0 = -1;
  for (size_t n = 0; n < 6; ++n) {
    if (faces[n].key < 0 || faces[n].key > 5) return "bad face key";
    byf[faces[n].key] = faces[n];
    if (faces[n].key == 0) first0 = int(n);
  }
  for (int t = 0; t < 6; ++t)
    if (faces[(first0 + t) % 6].key != t) return "faces are not in counter-clockwise index order";
  for (int f = 0; f < 6; ++f)
    for (auto& sl : byf[f].legs) {
      const Link& k = P->links[sl.first][sl.second];
      const Link& back = P->links[k.s2][k.l2];
      if (back.type != LINK_FACE || back.face != (f + 3) % 6)
        return "edges of a face must enter the opposite face";
    }
  P->faces.assign(1, byf);
  for (int f = 0; f < 6; ++f) P->msg_keys.push_back({f, -1});
  return "";
}

std::string sweep_schedule(const Problem& P, int block, int target,
                           const std::vector<int>& open_sites, Schedule* out) {
  const std::vector<int>& sites = P.blocks[block];
  const std::vector<Face>& F = P.faces[block];
  int nf = int(F.size());
  if (target < 0 || target >= nf) return "bad target face";
  std::set<int> inside(sites.begin(), sites.end());
  std::set<int> opens(open_sites.begin(), open_sites.end());
  std::vector<int64_t> chain;
  for (int k = 1; k < nf; ++k)
    for (auto& sl : F[(target + k) % nf].legs) chain.push_back(chain_in(sl.first, sl.second));
  std::set<std::pair<int, int>> tlegs(F[target].legs.begin(), F[target].legs.end());
  int64_t n = int64_t(sites.size()), sx = 0, sy = 0, fx = 0, fy = 0;
  for (int s : sites) { sx += P.sites[s].X; sy += P.sites[s].Y; }
  for (auto& sl : F[target].legs) {
    auto pt = P.leg_point(sl.first, sl.second);
    fx += pt.first; fy += pt.second;
  }
  int64_t k = int64_t(F[target].legs.size());
  int64_t dx = n * fx - 2 * k * sx, dy = n * fy - 2 * k * sy;
  std::set<int> remaining(sites.begin(), sites.end());
  out->steps.clear();
  while (!remaining.empty()) {
    std::map<int64_t, int> pos_of;
    for (size_t i = 0; i < chain.size(); ++i) pos_of[chain[i]] = int(i);
    bool found = false;
    int64_t bp = 0, bt = 0;
    int bs = -1, bpos = -1;
    std::vector<int> brun;
    for (int s : remaining) {
      int deg = P.sites[s].nslot;
      std::vector<int> ins;
      int p0 = int(chain.size());
      for (int l = 0; l < deg; ++l) {
        auto it = pos_of.find(chain_in(s, l));
        if (it != pos_of.end()) { ins.push_back(l); p0 = std::min(p0, it->second); }
      }
      if (ins.empty()) continue;
      int r = int(ins.size());
      bool ok = true;
      std::vector<int> run;
      for (int t = 0; t < r && ok; ++t) {
        int64_t id = chain[p0 + t];
        if (id < 0 || id / 8 != s) ok = false;
        else run.push_back(int(id % 8));
      }
      if (!ok) continue;
      for (int t = 0; t < r; ++t)
        if (run[t] != (run[0] + t) % deg) { ok = false; break; }
      if (!ok) continue;
      int64_t vx = n * 2 * P.sites[s].X - 2 * sx, vy = n * 2 * P.sites[s].Y - 2 * sy;
      int64_t kp = rdot(vx, vy, dx, dy), kt = rcross(vx, vy, dx, dy);
      if (!found || kp < bp || (kp == bp && kt < bt)) {
        found = true; bp = kp; bt = kt; bs = s; bpos = p0; brun = run;
      }
    }
    if (!found) return "no site can be swallowed with contiguous in-legs";
    int deg = P.sites[bs].nslot;
    int r = int(brun.size());
    Step st;
    st.site = bs;
    st.pos = bpos;
    st.in_slots = brun;
    for (int t = deg - r - 1; t >= 0; --t) st.out_slots.push_back((brun[0] + r + t) % deg);
    for (int l : st.out_slots) {
      if (tlegs.count({bs, l})) {
        st.out_ids.push_back(chain_out(bs, l));
      } else {
        const Link& lk = P.links[bs][l];
        if (lk.type != LINK_SITE || !inside.count(lk.s2))
          return "out-leg leaves the block off the target face";
        st.out_ids.push_back(chain_in(lk.s2, lk.l2));
      }
    }
    st.open = opens.count(bs) > 0;
    if (st.out_slots.empty()) {
      if (int(chain.size()) == r) return "chain would become empty";
      st.absorb = (bpos + r < int(chain.size())) ? 0 : 1;
    }
    chain.erase(chain.begin() + bpos, chain.begin() + bpos + r);
    chain.insert(chain.begin() + bpos, st.out_ids.begin(), st.out_ids.end());
    remaining.erase(bs);
    out->steps.push_back(st);
  }
  out->final_legs.clear();
  for (int64_t id : chain) {
    if (id >= 0) return "final chain is not the target face";
    int64_t c = -id - 1;
    out->final_legs.push_back({int(c / 8), int(c % 8)});
  }
  std::vector<std::pair<int, int>> a = out->final_legs, b = F[target].legs;
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  if (a != b) return "final chain misses target legs";
  return "";
}

}  // namespace pn

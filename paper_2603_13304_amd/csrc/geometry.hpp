// Kagome block geometry for the BlockBP engine: sites, legs, blocks, faces,
// face pairing of the self-messaging hexagonal block, and the order in which
// a boundary chain swallows a block.
//
// Lattice (Ch. "Block Belief Propagation", Sec. "Defining the Kagome block";
// App. "Kagome Block Indexing"): triangular Bravais lattice of up-triangles,
// cell R = i a1 + j a2, three sites per cell in the order Up, Down-Left,
// Down-Right; DL at R, DR at R + a1/2, U at R + a2/2.  Points are kept as
// integers (X, Y) with real position (X/4, sqrt(3) Y/4).
//
// Hexagonal block of face length N (3N^2-3N+1 cells, N_T = 3(3N^2-3N+1)
// sites) tiled by the superlattice V1 = N a1 + (N-1) a2 and its 60-degree
// rotations; face f is crossed by the edges that go into the copy at V_f and
// re-enter through face f+3 (Sec. "Conditions for studying infinite lattices
// using BlockBP").  Faces and the legs inside a face are ordered
// counter-clockwise starting from the bottom.
//
// Sweep order (the thesis shows it only in figures, Sec. "Contraction
// Order"): the chain starts as the incoming messages of all faces but the
// target, counter-clockwise after it; the next site is, among those whose
// chain legs form a contiguous run in the site's counter-clockwise leg order,
// the one with the smallest projection on the direction toward the target
// face's leg centroid (ties: transverse coordinate).
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace pn {

enum SiteKind { KIND_U = 0, KIND_DL = 1, KIND_DR = 2 };

struct Site {
  int ci = 0, cj = 0;     // cell
  int kind = 0;           // SiteKind
  int64_t X = 0, Y = 0;   // integer position
  int tensor = 0;         // index of the site's ket tensor
  int nslot = 4;
  int dirs[4] = {0, 0, 0, 0};  // bond direction (x 60 degrees) of each slot
};

enum LinkType { LINK_SITE = 0, LINK_OUTSIDE = 1, LINK_FACE = 2 };

struct Link {
  int type = LINK_OUTSIDE;
  int s2 = -1, l2 = -1;   // LINK_SITE: other end; LINK_FACE: periodic image
  int face = -1;          // LINK_FACE
};

enum FaceKey { FACE_BLOCK = 0, FACE_OUTSIDE = 1, FACE_HEX = 2 };

struct Face {
  int keytype = FACE_OUTSIDE;
  int key = -1;                          // neighbour block / hex face index / leg code
  std::vector<std::pair<int, int>> legs; // (site, slot) counter-clockwise
};

struct Step {
  int site = -1;
  int pos = 0;                  // chain index of the first in-leg
  std::vector<int> in_slots;    // chain order
  std::vector<int> out_slots;   // chain order
  std::vector<int64_t> out_ids; // chain leg ids replacing the run
  bool open = false;            // physical pair carried (expectation)
  int absorb = -1;              // out_slots empty: 0 = right neighbour, 1 = left
};

struct Schedule {
  std::vector<Step> steps;
  std::vector<std::pair<int, int>> final_legs;  // target legs in chain order
};

struct Problem {
  int kind = 0;  // 0 finite open patch, 1 infinite hexagonal block
  int N = 0, Lx = 0, Ly = 0, bLx = 0, bLy = 0;
  std::vector<Site> sites;
  std::vector<std::array<Link, 4>> links;
  std::vector<std::vector<int>> blocks;
  std::vector<int> block_of;
  std::vector<std::vector<Face>> faces;
  // directed messages: finite (a, b) = message a -> b; infinite (f, -1) =
  // message computed toward face f (stored on face f+3)
  std::vector<std::pair<int, int>> msg_keys;
  int V[6][2] = {};

  int n_tensors() const;
  std::pair<int64_t, int64_t> leg_point(int s, int l) const;  // twice the midpoint
  int face_index(int b, int keytype, int key) const;
  // message computed for msg_keys[m]: sending block, target face, and the
  // sender-side legs in the receiver's storage order
  void update_target(int m, int* block, int* face, std::vector<std::pair<int, int>>* recv) const;
  // storage slot (index into msg_keys of the stored message) feeding face f of block b; -1 = trivial
  int incoming_msg(int b, int f) const;
  // storage order legs of message slot m (receiver-side legs)
  const std::vector<std::pair<int, int>>& stored_legs(int m) const;
  int stored_slot_of_update(int m) const;   // where update m is stored
  std::vector<std::pair<int, int>> central_bonds() const;  // infinite only
  std::vector<std::pair<int, int>> bonds() const;          // finite internal bonds (s1 < s2)
};

// builders; return an empty string on success, else the error
std::string build_finite(Problem* P, int Lx, int Ly, int bLx, int bLy);
std::string build_hex(Problem* P, int N);
std::string sweep_schedule(const Problem& P, int block, int target,
                           const std::vector<int>& open_sites, Schedule* out);

inline int64_t chain_in(int s, int l) { return int64_t(s) * 8 + l; }
inline int64_t chain_out(int s, int l) { return -(int64_t(s) * 8 + l) - 1; }

}  // namespace pn

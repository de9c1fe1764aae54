// Marching-cubes case table, generated from a face-consistent rule.
//
// Marching cubes (Lorensen & Cline 1987) over the GLL sub-hexahedra; the
// paper renders such surfaces (section 4) without printing the method.  The
// 256-case table is built here from a rule, never copied from a published
// table.
//
// Corners v = a + 2b + 4c at (a, b, c).  Edge id = 4*axis + q, where q ranks
// the edge's lower corner among the four corners whose `axis` bit is 0.
//
// Face rule, in combinatorial form: walk the four corners of a face
// counter-clockwise as seen from outside the cube.  Each maximal run of
// above-isovalue corners is entered through one crossed edge and left
// through another; it contributes one segment from its leaving crossing to
// its entering crossing.  This keeps the above side on the left of the
// segment seen from outside, joins two crossings into one segment, and --
// on a face with four crossings -- gives each of the two diagonal above
// corners its own run, i.e. cuts the above corners apart.  Segments depend
// only on the face's four corner bits, so neighbouring cells agree on them.
//
// The segments form closed loops (every crossing lies on two faces).  Loops
// are listed by their smallest edge id; each is fan-triangulated along its
// orientation from the smallest edge id whose two faces contain no
// non-adjacent vertex of the same loop, which keeps every fan diagonal off
// the cube faces.  Triangles per case = crossed edges - 2 * loops.
#include <algorithm>
#include <cstring>
#include <vector>

#include "sem_internal.h"

namespace sem {
namespace {

struct Cube {
  int edge_lo[12], edge_hi[12], edge_axis[12];
  int face_ccw[6][4];        // corners, counter-clockwise seen from outside
  int face_edge[6][4];       // edge between face_ccw[f][q] and [q+1]
  bool edge_on_face[12][6];
};

int corner_bit(int v, int axis) { return (v >> axis) & 1; }

Cube make_cube() {
  Cube c;
  for (int axis = 0; axis < 3; ++axis) {
    int q = 0;
    for (int v = 0; v < 8; ++v) {
      if (corner_bit(v, axis)) continue;
      int e = 4 * axis + q++;
      c.edge_lo[e] = v;
      c.edge_hi[e] = v | (1 << axis);
      c.edge_axis[e] = axis;
    }
  }
  // Face (axis d, side s), f = 2d + s.  With (a, b) = the next two axes in
  // cyclic order, e_a x e_b = e_d: seen from +e_d the counter-clockwise
  // order in (a, b) is (0,0) (1,0) (1,1) (0,1); from -e_d it is reversed.
  for (int d = 0; d < 3; ++d) {
    int a = (d + 1) % 3, b = (d + 2) % 3;
    for (int s = 0; s < 2; ++s) {
      int f = 2 * d + s;
      int ab[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
      if (s == 0) std::swap(ab[1], ab[3]);
      for (int q = 0; q < 4; ++q)
        c.face_ccw[f][q] = (s << d) | (ab[q][0] << a) | (ab[q][1] << b);
    }
  }
  for (int f = 0; f < 6; ++f)
    for (int q = 0; q < 4; ++q) {
      int u = c.face_ccw[f][q], w = c.face_ccw[f][(q + 1) % 4];
      int lo = std::min(u, w), hi = std::max(u, w);
      for (int e = 0; e < 12; ++e)
        if (c.edge_lo[e] == lo && c.edge_hi[e] == hi) c.face_edge[f][q] = e;
    }
  for (int e = 0; e < 12; ++e)
    for (int f = 0; f < 6; ++f) {
      bool on = false;
      for (int q = 0; q < 4; ++q) on = on || c.face_edge[f][q] == e;
      c.edge_on_face[e][f] = on;
    }
  return c;
}

bool share_face(const Cube& c, int e1, int e2) {
  for (int f = 0; f < 6; ++f)
    if (c.edge_on_face[e1][f] && c.edge_on_face[e2][f]) return true;
  return false;
}

// Triangles of one case as edge triples, in slot order.
std::vector<int> case_triangles(const Cube& c, int cs) {
  int next[12];
  for (int e = 0; e < 12; ++e) next[e] = -1;
  for (int f = 0; f < 6; ++f) {
    bool up[4];
    for (int q = 0; q < 4; ++q) up[q] = (cs >> c.face_ccw[f][q]) & 1;
    for (int q = 0; q < 4; ++q) {
      // a run of above corners starts at q when corner q-1 is below
      if (!up[q] || up[(q + 3) % 4]) continue;
      int enter = c.face_edge[f][(q + 3) % 4];   // edge (q-1, q)
      int r = q;
      while (up[(r + 1) % 4]) r = (r + 1) % 4;
      int leave = c.face_edge[f][r];              // edge (r, r+1)
      next[leave] = enter;
    }
  }
  std::vector<int> tris;
  bool used[12] = {false};
  for (int start = 0; start < 12; ++start) {
    if (next[start] < 0 || used[start]) continue;
    std::vector<int> loop;
    for (int e = start; !used[e]; e = next[e]) {
      used[e] = true;
      loop.push_back(e);
    }
    const int n = (int)loop.size();
    int best = -1;
    for (int a = 0; a < n; ++a) {
      bool clash = false;
      for (int b = 0; b < n && !clash; ++b) {
        if (b == a || b == (a + 1) % n || b == (a + n - 1) % n) continue;
        clash = share_face(c, loop[a], loop[b]);
      }
      if (!clash && (best < 0 || loop[a] < loop[best])) best = a;
    }
    if (best < 0) best = 0;  // unreachable for the 256 cube cases
    for (int m = 1; m + 1 < n; ++m) {
      tris.push_back(loop[best]);
      tris.push_back(loop[(best + m) % n]);
      tris.push_back(loop[(best + m + 1) % n]);
    }
  }
  return tris;
}

}  // namespace

void build_mc_table(uint8_t* ntri, int8_t* tri) {
  const Cube c = make_cube();
  for (int cs = 0; cs < 256; ++cs) {
    std::vector<int> t = case_triangles(c, cs);
    const int nt = (int)t.size() / 3;
    if (ntri) ntri[cs] = (uint8_t)nt;
    if (tri) {
      for (int s = 0; s < kMcMaxTri * 3; ++s) tri[cs * kMcMaxTri * 3 + s] = -1;
      for (int s = 0; s < nt * 3 && s < kMcMaxTri * 3; ++s)
        tri[cs * kMcMaxTri * 3 + s] = (int8_t)t[s];
    }
  }
}

}  // namespace sem

// Switch function along chords of elements (Section 3, figure switchplt):
// host-side mesh preparation for meshes whose elements are oriented
// arbitrarily.  An element carries S^+_n on its face xi_n = 1 and -S^+_n on
// xi_n = 0; the two elements of a shared face carry opposite signs on it.  A
// chord is the path that enters an element through a face of direction n and
// leaves it through the other face of direction n.  Along a chord the sign
// seen on each face from the element being left is the same, so one choice
// per chord fixes all of it; every (element, direction) lies on one chord.
// Chords are started in element order, then local-direction order, with
// S^+ = +1 at the start, and walked both ways to a boundary or back to the
// start.
#include <string>
#include <vector>

#include "ldg_ctx.hpp"

namespace {

// node at the xi_n = s end of face line l (other coordinates in increasing
// dimension order, lowest fastest)
int end_node(int D, int N1, int n, int l, int s) {
  int node = 0, mul = 1, rem = l;
  for (int d = 0; d < D; ++d) {
    int c;
    if (d == n) {
      c = s ? N1 - 1 : 0;
    } else {
      c = rem % N1;
      rem /= N1;
    }
    node += c * mul;
    mul *= N1;
  }
  return node;
}

// if node lies on face xi_n = s, its face line index; else -1
int face_line(int D, int N1, int node, int n, int s) {
  int l = 0, mul = 1;
  for (int d = 0; d < D; ++d) {
    const int c = node % N1;
    node /= N1;
    if (d == n) {
      if (c != (s ? N1 - 1 : 0)) return -1;
    } else {
      l += c * mul;
      mul *= N1;
    }
  }
  return l;
}

}  // namespace

extern "C" {

ldg_status ldg_assign_switches(int32_t dim, int32_t p, int64_t n_elem, const int64_t* face_nbr_host,
                               const int32_t* nbr_node_host, int8_t* switch_plus_host) {
  const int D = dim, N1 = p + 1;
  if (dim < 2 || dim > 3 || p < 1 || n_elem < 1 || !face_nbr_host || !nbr_node_host || !switch_plus_host) {
    ldg_host::set_host_error("ldg_assign_switches: bad dimension, degree, element count or null pointer");
    return LDG_E_INVALID;
  }
  int NL = 1;
  for (int d = 1; d < D; ++d) NL *= N1;
  const int64_t E = n_elem;
  std::vector<int8_t> S((size_t)E * D, 0);
  auto reverse_face = [&](int64_t e, int f, int64_t nb) -> int {
    // the neighbour's face that coincides with face f of e, found through the node maps
    const int mine = end_node(D, N1, f / 2, 0, f % 2);
    const int theirs = nbr_node_host[(e * 2 * D + f) * NL + 0];
    for (int f2 = 0; f2 < 2 * D; ++f2) {
      if (face_nbr_host[nb * 2 * D + f2] != e) continue;
      const int l2 = face_line(D, N1, theirs, f2 / 2, f2 % 2);
      if (l2 < 0) continue;
      if (nbr_node_host[(nb * 2 * D + f2) * NL + l2] == mine) return f2;
    }
    return -1;
  };
  for (int64_t e0 = 0; e0 < E; ++e0)
    for (int n0 = 0; n0 < D; ++n0) {
      if (S[e0 * D + n0]) continue;
      S[e0 * D + n0] = 1;
      for (int start = 1; start >= 0; --start) {
        int64_t e = e0;
        int n = n0, side = start;
        for (;;) {
          const int f = 2 * n + side;
          const int64_t nb = face_nbr_host[e * 2 * D + f];
          if (nb < 0) break;
          if (nb >= E) {
            ldg_host::set_host_error("ldg_assign_switches: neighbour index out of range (element " +
                                     std::to_string(e) + ", face " + std::to_string(f) + ")");
            return LDG_E_SHAPE;
          }
          const int f2 = reverse_face(e, f, nb);
          if (f2 < 0) {
            ldg_host::set_host_error("ldg_assign_switches: face connectivity is not reciprocal (element " +
                                     std::to_string(e) + ", face " + std::to_string(f) + ")");
            return LDG_E_SHAPE;
          }
          // sign on the shared face seen from e; the neighbour must show the opposite
          const int here = side ? S[e * D + n] : -S[e * D + n];
          const int8_t want = (int8_t)((f2 % 2) ? -here : here);
          int8_t& t = S[nb * D + f2 / 2];
          if (t) {
            if (t != want) {
              ldg_host::set_host_error("ldg_assign_switches: a chord returns with the opposite sign (element " +
                                       std::to_string(nb) + ")");
              return LDG_E_SHAPE;
            }
            break;
          }
          t = want;
          e = nb;
          n = f2 / 2;
          side = 1 - f2 % 2;
        }
      }
    }
  for (size_t i = 0; i < S.size(); ++i) switch_plus_host[i] = S[i];
  return LDG_OK;
}

}  // extern "C"

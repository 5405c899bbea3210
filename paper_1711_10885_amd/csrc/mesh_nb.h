// Face neighbours on the tensor grid, with optional periodic axes.
#pragma once

#include <hip/hip_runtime.h>

namespace dgmf {

// Neighbour across the face of a cell (index ia of na along axis a, cell
// stride cst along a) on side e (0: lower, 1: upper).  On a periodic axis the
// first and last cells are neighbours across the domain boundary (`wrap`);
// otherwise a face on the domain boundary has no neighbour (in = false, the
// homogeneous Dirichlet case) and cell/ja repeat the cell's own.
struct FaceNb {
  bool in;
  bool wrap;
  int ja;
  int cell;
};

__host__ __device__ __forceinline__ FaceNb face_nb(int cell, int ia, int na, int cst, bool periodic, int e) {
  FaceNb r;
  if (e) {
    r.wrap = periodic && ia + 1 == na;
    r.in = ia + 1 < na || r.wrap;
    r.ja = r.wrap ? 0 : ia + 1;
  } else {
    r.wrap = periodic && ia == 0;
    r.in = ia > 0 || r.wrap;
    r.ja = r.wrap ? na - 1 : ia - 1;
  }
  if (!r.in) r.ja = ia;
  r.cell = cell + (r.ja - ia) * cst;
  return r;
}

// Node of axis a at which b_a is read on face (ia, e): the face's own node,
// except that the face across a periodic boundary uses node 0 from both
// sides, so that both cells see the same normal velocity.
__host__ __device__ __forceinline__ int face_node(int ia, int e, bool wrap) { return (e && wrap) ? 0 : ia + e; }

}  // namespace dgmf

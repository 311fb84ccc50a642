// Stencil tables of the 3D Jacobian (slot layout of include/acch.h).
#pragma once

#include "common.h"

namespace acch {

constexpr int kNSlot3D = 40;

struct Off3 {
  int dx, dy, dz;
};

// u-row/u-col offsets: the cell, the 6 faces (-x,+x,-y,+y,-z,+z), the 6 second
// neighbours along the axes, and the 12 edge neighbours.
__host__ __device__ constexpr Off3 uu3(int k) {
  constexpr Off3 t[25] = {{0, 0, 0},   {-1, 0, 0},  {1, 0, 0},   {0, -1, 0},  {0, 1, 0},  {0, 0, -1}, {0, 0, 1},
                          {-2, 0, 0},  {2, 0, 0},   {0, -2, 0},  {0, 2, 0},   {0, 0, -2}, {0, 0, 2},  {-1, -1, 0},
                          {1, -1, 0},  {-1, 1, 0},  {1, 1, 0},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1}, {1, 0, 1},
                          {0, -1, -1}, {0, 1, -1},  {0, -1, 1},  {0, 1, 1}};
  return t[k];
}
// the cell and its 6 faces (u-row/v-col, v-row/v-col)
__host__ __device__ constexpr Off3 star3(int k) {
  constexpr Off3 t[7] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  return t[k];
}

}  // namespace acch

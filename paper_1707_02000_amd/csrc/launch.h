// Launch sizes for the grid-stride kernels of the graph passes (k-truss listing,
// core numbers, reordering, h-index iteration).
#pragma once
#include "common.h"

// Workgroups for `count` items, one per lane; the kernels stride over the rest.
static inline int grid_items(i64 count, int cap = 8192) {
  i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Workgroups for `count` items, one per wave; the kernels stride over the rest.
static inline int grid_waves(i64 count, int cap = 8192) {
  const i64 waves = PKT_BLOCK / PKT_WAVE;
  i64 g = (count + waves - 1) / waves;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

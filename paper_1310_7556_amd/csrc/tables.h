// Host FP64 tables of the track finder (see tables.cpp).
#pragma once

#include "../../include/hough.h"

namespace hough {

constexpr uint32_t kMaxLayers = 16;

bool spec_valid(const hough_grid_spec &g);
void build_offsets(const hough_grid_spec &g, uint32_t *O, uint8_t *V);
void build_zshift(const hough_grid_spec &g, int32_t *Z);

}  // namespace hough

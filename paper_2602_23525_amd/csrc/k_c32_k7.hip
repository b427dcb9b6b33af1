// Tile-kernel variant: float complex, kernel kind 7 (see tile.h), up to 16
// elements per thread.
#include "tile_launch.h"

MFFT_TILE_LAUNCHERS(float, c32_k7, 7)

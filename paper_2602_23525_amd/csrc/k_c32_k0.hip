// Tile-kernel variant: float complex, kernel kind 0 (see tile.h), up to 16
// elements per thread.
#include "tile_launch.h"

MFFT_TILE_LAUNCHERS(float, c32_k0, 0)

// Tile-kernel variant: double complex, kernel kind 7 (see tile.h), up to 16
// elements per thread.
#include "tile_launch.h"

MFFT_TILE_LAUNCHERS(double, c64_k7, 7)

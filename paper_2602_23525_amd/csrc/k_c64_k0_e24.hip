// Tile-kernel variant: double complex, kernel kind 0 (see tile.h), up to 24
// elements per thread, for lines whose radices include 17, 19 or 23.
#include "tile_launch.h"

MFFT_TILE_LAUNCHERS_E(double, c64_k0_e24, 0, 24)

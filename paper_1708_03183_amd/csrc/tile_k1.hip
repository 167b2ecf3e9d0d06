// Tile kernels of the P1 element.
#define DGT_TILE_K 1
#include "tile_launch_impl.h"

// Tile kernels of the P3 element.
#define DGT_TILE_K 3
#include "tile_launch_impl.h"

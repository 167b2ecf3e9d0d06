// Tile kernels of the P2 element.
#define DGT_TILE_K 2
#include "tile_launch_impl.h"

// Tile kernels of the P4 element.
#define DGT_TILE_K 4
#include "tile_launch_impl.h"

// Walled passes with complex float propagators.
#define PFT_WALLS_T float
#include "passes_walls.inc"

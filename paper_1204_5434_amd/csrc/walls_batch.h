// Batched walled passes: the walled z and strided passes over the replicas of
// one batch group (one grid and one set of walls), blockIdx.y selecting a
// replica whose arguments come from a device table (skip: no work at this
// sweep position).  Every axis length uses its default radix split and tile,
// so a table's strided ntiles must be spass_tiles(n, 0, ncols).
#pragma once

#include "kernels.h"

namespace pft {

template <typename T>
hipError_t launch_zpass_walls_batch(int nz, int ext, int64_t nlines, const ZArgs<T>* descs, int nrep, hipStream_t s);
template <typename T>
hipError_t launch_spass_walls_batch(int axis, int n, int ext, int64_t ncols, int nslabs, const SArgs<T>* descs,
                                    int nrep, hipStream_t s);

}  // namespace pft

// complex128 instantiations of the fused tile pass with the per-tile read-out
#include "tile_kernel.cuh"

namespace qsim {
void launch_tile_f64_z(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, double *zparts, hipStream_t st)
{
    launch_tile_t<double, 2>(a, n_tiles, log_r, log_nt, zparts, st);
}
}  // namespace qsim

// complex64 instantiations of the fused tile pass
#include "tile_kernel.cuh"

namespace qsim {
void launch_tile_f32(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st)
{
    launch_tile_t<float>(a, n_tiles, log_r, log_nt, st);
}
}  // namespace qsim

// complex64 instantiations of the fused tile pass with plain loads and stores
#include "tile_kernel.cuh"

namespace qsim {
void launch_tile_f32_plain(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st)
{
    launch_tile_t<float, 0>(a, n_tiles, log_r, log_nt, nullptr, st);
}
}  // namespace qsim

// complex128 instantiations of the fused tile pass over whole 128-byte lines
// (non-temporal access); other passes go to launch_tile_f64_plain
#include "kernels.h"
#include "tile_kernel.cuh"

namespace qsim {
void launch_tile_f64(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st)
{
    if (a.io & 8u)
        launch_tile_t<double, 1>(a, n_tiles, log_r, log_nt, nullptr, st);
    else
        launch_tile_f64_plain(a, n_tiles, log_r, log_nt, st);
}
}  // namespace qsim

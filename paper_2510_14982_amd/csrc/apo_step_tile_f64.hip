// apo_step_tile_f64.hip -- tiled (LDS + MFMA / histogram tables) step kernels, binary64.
#include "apo_step.hpp"

namespace apok {

hipError_t launch_tile_f64(const Params &p, int init, hipStream_t s) {
    return p.np == 1 ? launch_tile_t<double, 1>(p, init, s) : launch_tile_t<double, kMaxNp>(p, init, s);
}

hipError_t launch_tile_batch_f64(const Params &proto, const BatchLaunch &b, hipStream_t s) {
    return proto.np == 1 ? launch_tile_t<double, 1>(proto, 0, s, &b)
                         : launch_tile_t<double, kMaxNp>(proto, 0, s, &b);
}

hipError_t launch_tile_persist_f64(const Params &p, int t0, int n, hipStream_t s) {
    return p.np == 1 ? launch_tile_persist_t<double, 1>(p, t0, n, s)
                     : launch_tile_persist_t<double, kMaxNp>(p, t0, n, s);
}

}  // namespace apok

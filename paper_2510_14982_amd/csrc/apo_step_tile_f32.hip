// apo_step_tile_f32.hip -- tiled (LDS + MFMA / histogram tables) step kernels, binary32.
#include "apo_step.hpp"

namespace apok {

hipError_t launch_tile_f32(const Params &p, int init, hipStream_t s) {
    return p.np == 1 ? launch_tile_t<float, 1>(p, init, s) : launch_tile_t<float, kMaxNp>(p, init, s);
}

hipError_t launch_tile_batch_f32(const Params &proto, const BatchLaunch &b, hipStream_t s) {
    return proto.np == 1 ? launch_tile_t<float, 1>(proto, 0, s, &b)
                         : launch_tile_t<float, kMaxNp>(proto, 0, s, &b);
}

hipError_t launch_tile_persist_f32(const Params &p, int t0, int n, hipStream_t s) {
    return p.np == 1 ? launch_tile_persist_t<float, 1>(p, t0, n, s)
                     : launch_tile_persist_t<float, kMaxNp>(p, t0, n, s);
}

}  // namespace apok

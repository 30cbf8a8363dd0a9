// CPU check of the step kernels' launch shapes (apo_shape.hpp, the header
// the library itself uses): for every dimension and every lane count a
// policy can give, prints what the library would launch and whether that
// shape is compiled and fits the LDS.  Output, one line per case:
//   S es dim G NCH TM built fits key decoded_G decoded_NCH decoded_TM
// then, for the batch policy (rotated; separable or Rosenbrock):
//   P es dim rosenbrock G NCH TM fits
// then, for the persistent elementwise form at its largest population
// (256 / G protozoa), the LDS image of the run and its regions' offsets:
//   I es dim G pop bytes x0 x1 f fs perm drf pdr lb ub sh
#include <cstdio>

#include "apo_shape.hpp"

using namespace apok;

int main() {
    const int lanes[] = {4, 8, 16, 32, 64};
    for (int es = 4; es <= 8; es += 4)
        for (int dim = 1; dim <= 1024; ++dim)
            for (int G : lanes)
                for (int wide = 0; wide < 2; ++wide) {
                    const int NCH = chunks_for(dim, G);
                    const int TM = wide ? tile_rows_wide(G) : 16;
                    const bool built = NCH > 0 && tile_shape_built(G, NCH, TM);
                    const bool fits = NCH > 0 && tile_shape_ok(dim, G, NCH, TM, es);
                    const int key = NCH > 0 ? pack_shape(es == 8, true, true, G, NCH, TM) : -1;
                    const int kg = key < 0 ? -1 : (key >> 3) & 0xFF;
                    const int kc = key < 0 ? -1 : (key >> 11) & 0xF;
                    const int kt = key < 0 ? -1 : (key >> 15) & 0x1FF;
                    std::printf("S %d %d %d %d %d %d %d %d %d %d %d\n", es, dim, G, NCH, TM,
                                built ? 1 : 0, fits ? 1 : 0, key, kg, kc, kt);
                }
    for (int es = 4; es <= 8; es += 4)
        for (int dim = 1; dim <= 1024; ++dim)
            for (int ros = 0; ros < 2; ++ros) {
                const int lanes = batch_lanes(dim, true, ros != 0, es);
                const int G = lanes ? lanes : lanes_for_dim(dim);
                const int NCH = chunks_for(dim, G), TM = tile_rows_wide(G);
                const bool fits = NCH > 0 && tile_shape_ok(dim, G, NCH, TM, es);
                std::printf("P %d %d %d %d %d %d %d\n", es, dim, ros, G, NCH, TM, fits ? 1 : 0);
            }
    for (int es = 4; es <= 8; es += 4)
        for (int dim = 1; dim <= 1024; ++dim) {
            const int G = lanes_for_dim(dim), pop = 256 / G;
            const PersistImage m = persist_image(pop, row_stride(dim, es), es, false);
            std::printf("I %d %d %d %d %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", es, dim, G,
                        pop, m.total, m.x0, m.x1, m.f, m.fs, m.perm, m.drf, m.pdr, m.lb, m.ub,
                        m.sh);
        }
    return 0;
}

// Host check of the workgroup-order maps of dev_common.h: xcd_stretch is a bijection of
// [0, G), and xcd_tile a bijection of [0, B T) onto (right-hand side, tile) pairs, for
// batch sizes, tile counts and groupings that include partial stretches and groups.
// Prints "ok" and exits 0, or prints the first failing case and exits 1.
#include <cstdio>
#include <vector>

#include "dev_common.h"

int main() {
  for (unsigned G = 1; G <= 4000; G += (G < 64 ? 1 : 37)) {
    std::vector<int> seen(G, 0);
    for (unsigned id = 0; id < G; ++id) {
      const unsigned l = xcd_stretch(id, G);
      if (l >= G || seen[l]++) {
        std::printf("xcd_stretch G=%u id=%u -> %u\n", G, id, l);
        return 1;
      }
    }
    // equal stretches: ids of one XCD map to consecutive positions
    for (unsigned id = HELM_XCDS; id < G; ++id)
      if (xcd_stretch(id, G) != xcd_stretch(id - HELM_XCDS, G) + 1) {
        std::printf("xcd_stretch G=%u id=%u: not contiguous\n", G, id);
        return 1;
      }
  }
  for (unsigned B : {1u, 3u, 7u, 8u, 15u, 60u, 61u})
    for (unsigned T : {1u, 5u, 37u, 490u})
      for (unsigned g : {0u, 1u, 4u, 16u, 60u}) {
        std::vector<int> seen(B * T, 0);
        for (unsigned id = 0; id < B * T; ++id) {
          const TileId o = xcd_tile(id, B, T, g);
          if (o.b < 0 || o.b >= (int)B || o.t < 0 || o.t >= (int)T || seen[o.b * T + o.t]++) {
            std::printf("xcd_tile B=%u T=%u g=%u id=%u -> (%d, %d)\n", B, T, g, id, o.b, o.t);
            return 1;
          }
        }
      }
  std::printf("ok\n");
  return 0;
}

// The fused chemistry-update kernel instantiated for FP16 operands.
#include "step_kernel.h"

namespace chemdnn {

// Compiled network shapes: the 17-species net (400, 200, 100) and the
// 29-species net (1600, 800, 400).
bool find_layout_fp16(int h1, int h2, int h3, NetLayout *out) {
  if (h1 == 400 && h2 == 200 && h3 == 100) {
    fill_layout<Cfg<OpF16, 4, 4, 400, 200, 100>, false>(out);
    return true;
  }
  if (h1 == 1600 && h2 == 800 && h3 == 400) {
    fill_layout<Cfg<OpF16, 4, 8, 1600, 800, 400>, false>(out);
    return true;
  }
  return false;
}

// Property mode: the density network of the supercritical flame,
// 3-1024-512-256-1 (its 1.35 MB of BF16 weights fit the L2 of an XCD).
bool find_prop_layout_fp16(int h1, int h2, int h3, NetLayout *out) {
  if (h1 == 1024 && h2 == 512 && h3 == 256) {
    fill_prop_layout<Cfg<OpF16, 4, 8, 1024, 512, 256>>(out);
    return true;
  }
  return false;
}

}  // namespace chemdnn

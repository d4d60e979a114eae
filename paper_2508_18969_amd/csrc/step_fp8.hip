// The fused chemistry-update kernel instantiated for FP8 E4M3 operands.
#include "step_kernel.h"

namespace chemdnn {

// Compiled network shapes: the 17-species net (400, 200, 100) and the
// 29-species net (1600, 800, 400).
bool find_layout_fp8(int h1, int h2, int h3, NetLayout *out) {
  if (h1 == 400 && h2 == 200 && h3 == 100) {
    fill_layout<Cfg<OpF8, 3, 4, 400, 200, 100>, false>(out);
    return true;
  }
  if (h1 == 1600 && h2 == 800 && h3 == 400) {
    fill_layout<Cfg<OpF8, 4, 8, 1600, 800, 400>, false>(out);
    return true;
  }
  return false;
}

}  // namespace chemdnn

// Contraction kernels specialised for l_a + l_b = 2 (all l_c + l_d, I1-I6), FP64.
#include "f12_big.h"

namespace f12 {

int launch_big_lab2(int lcd, int i5, const ContractArgs &a, unsigned nblocks, hipStream_t st) {
  return launch_big_lab<2, 0>(lcd, i5, a, nblocks, st);
}

}  // namespace f12

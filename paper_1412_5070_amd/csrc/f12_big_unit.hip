// The contraction kernels of f12_big.h for one value of l_a + l_b (F12_LAB,
// all l_c + l_d, I1-I6) and one ket-transform precision (F12_PREC: 0 FP64,
// 1 split FP32).  The build compiles this file once per pair so that the
// shape instantiations compile in parallel.
#include "f12_big.h"

#if !defined(F12_LAB) || !defined(F12_PREC)
#error "build with -DF12_LAB=<0..6> -DF12_PREC=<0|1>"
#endif

namespace f12 {

template <int LAB, int PREC>
int launch_big_unit(int lcd, int i5, const ContractArgs &a, unsigned nblocks, hipStream_t st);

template <>
int launch_big_unit<F12_LAB, F12_PREC>(int lcd, int i5, const ContractArgs &a, unsigned nblocks,
                                       hipStream_t st) {
  return launch_big_lab<F12_LAB, F12_PREC>(lcd, i5, a, nblocks, st);
}

}  // namespace f12

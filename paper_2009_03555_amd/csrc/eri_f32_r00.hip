// ERI + digest kernels of bra pair class 0, ket pair class 0: FP32 recursion and
// primitive sum (mixed precision), FP64 ladder, HRR and digest.
#include "eri_kernels.hpp"
HFX_ERI_F32_UNIT(0, 0)

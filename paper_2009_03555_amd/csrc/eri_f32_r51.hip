// ERI + digest kernels of bra pair class 5, ket pair class 1: FP32 recursion and
// primitive sum (mixed precision), FP64 ladder, HRR and digest.
#include "eri_kernels.hpp"
HFX_ERI_F32_UNIT(5, 1)

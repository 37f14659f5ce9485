// ERI + digest kernels of bra pair class 1, ket pair class 0.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(1, 0)

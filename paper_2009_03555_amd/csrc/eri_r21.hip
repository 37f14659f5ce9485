// ERI + digest kernels of bra pair class 2, ket pair class 1.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(2, 1)

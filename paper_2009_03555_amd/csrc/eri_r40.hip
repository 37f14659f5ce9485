// ERI + digest kernels of bra pair class 4, ket pair class 0.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(4, 0)

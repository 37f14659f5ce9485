// ERI + digest kernels of bra pair class 5, ket pair class 4.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(5, 4)

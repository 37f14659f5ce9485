// ERI + digest kernels of bra pair class 1, ket pair class 1.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(1, 1)
HFX_SCHWARZ_UNIT(1)

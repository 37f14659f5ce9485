// ERI + digest kernels of bra pair class 3, ket pair class 3.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(3, 3)
HFX_SCHWARZ_UNIT(3)

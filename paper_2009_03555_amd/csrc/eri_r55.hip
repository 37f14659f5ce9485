// ERI + digest kernels of bra pair class 5, ket pair class 5.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(5, 5)
HFX_SCHWARZ_UNIT(5)

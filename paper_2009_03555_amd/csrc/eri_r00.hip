// ERI + digest kernels of bra pair class 0, ket pair class 0.
#include "eri_kernels.hpp"
HFX_ERI_UNIT(0, 0)
HFX_SCHWARZ_UNIT(0)

// Wave-cooperative ERI + digest kernel of bra pair class 4, ket pair class 3.
#include "eri_coop.hpp"
HFX_COOP_UNIT(4, 3)

// Wave-cooperative ERI + digest kernel of bra pair class 5, ket pair class 4.
#include "eri_coop.hpp"
HFX_COOP_UNIT(5, 4)

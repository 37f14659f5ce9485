// Schwarz factors of pair class 5 by the wave-cooperative kernel.
#include "eri_coop.hpp"
HFX_COOP_SCHWARZ_UNIT(5)

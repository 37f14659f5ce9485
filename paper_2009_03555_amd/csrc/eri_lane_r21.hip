// Lane-per-component ERI + digest kernels (FP64 and FP32) of bra pair class 2, ket pair class 1.
#include "eri_lane.hpp"
HFX_LANE_UNIT(2, 1)

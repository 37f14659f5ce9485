// Lane-per-component ERI + digest kernels (FP64 and FP32) of bra pair class 3, ket pair class 3.
#include "eri_lane.hpp"
HFX_LANE_UNIT(3, 3)

// Lane-per-component ERI + digest kernels (FP64 and FP32) of bra pair class 4, ket pair class 0.
#include "eri_lane.hpp"
HFX_LANE_UNIT(4, 0)

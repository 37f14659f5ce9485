// Lane-per-component ERI + digest kernels (FP64 and FP32) of bra pair class 5, ket pair class 0.
#include "eri_lane.hpp"
HFX_LANE_UNIT(5, 0)

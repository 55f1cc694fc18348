// MT predictor-flux kernel instantiations for the FP32 working precision.
#include "ctu_dispatch.hpp"
CTU_DEFINE_MT_DISPATCH(float, f32)

// MT predictor-flux kernel instantiations for the FP64 working precision.
#include "ctu_dispatch.hpp"
CTU_DEFINE_MT_DISPATCH(double, f64)

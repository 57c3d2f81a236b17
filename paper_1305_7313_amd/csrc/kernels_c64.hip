// FP32 (complex64) instantiations.
#define FX_T float
#include "launch_impl.h"

// FP64 (complex128) instantiations.
#define FX_T double
#include "launch_impl.h"

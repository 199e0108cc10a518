// kernels_small.hip -- placeholder translation unit for the small-state loop.
#include "internal.h"

// Launchers and kernels of one scheme (SWEPT_SCHEME, set by the build: one
// object per scheme, compiled in parallel).
#include "stages.hpp"

#ifndef SWEPT_SCHEME
#error "build with -DSWEPT_SCHEME=<scheme struct>"
#endif

template struct swept::Stages<swept::SWEPT_SCHEME>;

// The Barnes-Hut kernels with the field gradient (bh_kernel.h), compiled
// apart from the others so that the two halves build in parallel.
#include "bh_kernel.h"

bh_fn bh_select_grad(int s, int p, bool f32, bool h) { return bh_select<true>(s, p, f32, h); }

// The near-field kernels (p2p_kernel.h) for charges, dipoles and quadrupoles (masks 1-7).
#include "p2p_kernel.h"

bool p2p_dispatch_lo(int mask, bool f32, bool grad, unsigned nblocks, hipStream_t s, const P2PArgs &a)
{
    switch (mask) {
    case 1: p2p_launch_mask<1>(f32, grad, nblocks, s, a); return true;
    case 2: p2p_launch_mask<2>(f32, grad, nblocks, s, a); return true;
    case 3: p2p_launch_mask<3>(f32, grad, nblocks, s, a); return true;
    case 4: p2p_launch_mask<4>(f32, grad, nblocks, s, a); return true;
    case 5: p2p_launch_mask<5>(f32, grad, nblocks, s, a); return true;
    case 6: p2p_launch_mask<6>(f32, grad, nblocks, s, a); return true;
    case 7: p2p_launch_mask<7>(f32, grad, nblocks, s, a); return true;
    default: return false;
    }
}

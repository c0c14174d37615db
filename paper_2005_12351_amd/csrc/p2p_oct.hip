// The near-field kernels (p2p_kernel.h) for systems with octupoles (masks 8-15).
#include "p2p_kernel.h"

bool p2p_dispatch_oct(int mask, bool f32, bool grad, unsigned nblocks, hipStream_t s, const P2PArgs &a)
{
    switch (mask) {
    case 8: p2p_launch_mask<8>(f32, grad, nblocks, s, a); return true;
    case 9: p2p_launch_mask<9>(f32, grad, nblocks, s, a); return true;
    case 10: p2p_launch_mask<10>(f32, grad, nblocks, s, a); return true;
    case 11: p2p_launch_mask<11>(f32, grad, nblocks, s, a); return true;
    case 12: p2p_launch_mask<12>(f32, grad, nblocks, s, a); return true;
    case 13: p2p_launch_mask<13>(f32, grad, nblocks, s, a); return true;
    case 14: p2p_launch_mask<14>(f32, grad, nblocks, s, a); return true;
    case 15: p2p_launch_mask<15>(f32, grad, nblocks, s, a); return true;
    default: return false;
    }
}

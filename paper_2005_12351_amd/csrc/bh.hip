// Barnes-Hut evaluation of potential and field (the kernel is in
// bh_kernel.h; its instantiations, with and without the field gradient, per
// source order, are generated translation units, gen_bh.py).
#include "bh_kernel.h"

static bh_fn bh_select(bool grad, int s, int p, bool f32, bool h)
{
    switch (s) {
    case 0: return grad ? bh_select_g_s0(p, f32, h) : bh_select_f_s0(p, f32, h);
    case 1: return grad ? bh_select_g_s1(p, f32, h) : bh_select_f_s1(p, f32, h);
    case 2: return grad ? bh_select_g_s2(p, f32, h) : bh_select_f_s2(p, f32, h);
    case 3: return grad ? bh_select_g_s3(p, f32, h) : bh_select_f_s3(p, f32, h);
    default: return nullptr;
    }
}

namespace {

// counters are cleared by a kernel, not a memset, so that the launch
// sequence can be captured into a graph
__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_bh(fmm_tree *t, int outputs, double *phi, double *field, double *grad, hipStream_t s)
{
    const bool f32 = t->prec == FMM_PREC_MIXED, h = t->basis == FMM_M2L_HARMONIC;
    bh_fn k = bh_select((outputs & FMM_GRAD) != 0, t->order, t->p, f32, h);
    if (!k) return hipErrorInvalidValue;
    BHArgs a;
    a.cells = t->d_cells;
    a.xs = t->d_x;
    a.m64 = t->d_mom;
    a.m32 = t->d_mom32;
    a.M = h ? (const void *)t->d_Mh : (f32 ? (const void *)t->d_M32 : (const void *)t->d_M64);
    a.perm = t->d_perm;
    a.phi = phi;
    a.field = field;
    a.n = (int)t->ht.n;
    a.nmp = h ? (hterms(t->p) - hterms(t->order - 1) + 3) / 4 * 4 : (nterms(t->p) - nterms(t->order - 1) + 3) / 4 * 4;
    a.outputs = outputs;
    a.theta2 = t->theta * t->theta;
    for (int d = 0; d < 3; ++d) a.g.lo[d] = t->ht.lo[d];
    a.g.h = t->ht.h;
    a.counts = t->d_bhcount;
    a.mask = t->smask;
    a.w = mask_width(t->smask);
    a.grad = grad;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, t->d_bhcount, 2);
    hipLaunchKernelGGL(k, dim3((unsigned)((t->ht.n + 63) / 64)), dim3(64), 0, s, a);
    return hipGetLastError();
}

// Selects the generated M2L kernel for (p, s, precision, basis), s = 0..3.
#include "fmm_internal.h"

bool m2l_lookup_s0_f32(int p, M2LVariant *v);
bool m2l_lookup_s1_f32(int p, M2LVariant *v);
bool m2l_lookup_s2_f32(int p, M2LVariant *v);
bool m2l_lookup_s0_f64(int p, M2LVariant *v);
bool m2l_lookup_s1_f64(int p, M2LVariant *v);
bool m2l_lookup_s2_f64(int p, M2LVariant *v);
bool m2l_lookup_s0_f32_h(int p, M2LVariant *v);
bool m2l_lookup_s1_f32_h(int p, M2LVariant *v);
bool m2l_lookup_s2_f32_h(int p, M2LVariant *v);
bool m2l_lookup_s0_f64_h(int p, M2LVariant *v);
bool m2l_lookup_s1_f64_h(int p, M2LVariant *v);
bool m2l_lookup_s2_f64_h(int p, M2LVariant *v);
bool m2l_lookup_s0_f32_hm(int p, M2LVariant *v);
bool m2l_lookup_s1_f32_hm(int p, M2LVariant *v);
bool m2l_lookup_s2_f32_hm(int p, M2LVariant *v);
bool m2l_lookup_s3_f32(int p, M2LVariant *v);
bool m2l_lookup_s3_f64(int p, M2LVariant *v);
bool m2l_lookup_s3_f32_h(int p, M2LVariant *v);
bool m2l_lookup_s3_f64_h(int p, M2LVariant *v);
bool m2l_lookup_s3_f32_hm(int p, M2LVariant *v);

bool m2l_lookup(int p, int s, bool fp32, bool harmonic, M2LVariant *v, bool mfma)
{
    if (harmonic && fp32 && mfma) {
        switch (s) {
        case 0: return m2l_lookup_s0_f32_hm(p, v);
        case 1: return m2l_lookup_s1_f32_hm(p, v);
        case 2: return m2l_lookup_s2_f32_hm(p, v);
        case 3: return m2l_lookup_s3_f32_hm(p, v);
        default: return false;
        }
    }
    if (harmonic) {
        switch (s) {
        case 0: return fp32 ? m2l_lookup_s0_f32_h(p, v) : m2l_lookup_s0_f64_h(p, v);
        case 1: return fp32 ? m2l_lookup_s1_f32_h(p, v) : m2l_lookup_s1_f64_h(p, v);
        case 2: return fp32 ? m2l_lookup_s2_f32_h(p, v) : m2l_lookup_s2_f64_h(p, v);
        case 3: return fp32 ? m2l_lookup_s3_f32_h(p, v) : m2l_lookup_s3_f64_h(p, v);
        default: return false;
        }
    }
    switch (s) {
    case 0: return fp32 ? m2l_lookup_s0_f32(p, v) : m2l_lookup_s0_f64(p, v);
    case 1: return fp32 ? m2l_lookup_s1_f32(p, v) : m2l_lookup_s1_f64(p, v);
    case 2: return fp32 ? m2l_lookup_s2_f32(p, v) : m2l_lookup_s2_f64(p, v);
    case 3: return fp32 ? m2l_lookup_s3_f32(p, v) : m2l_lookup_s3_f64(p, v);
    default: return false;
    }
}

// Launchers of the even-odd Dslash for every link storage format.
#pragma once

#include "common.h"

namespace stag {

// The operator's link copies.  d18 is the master FP64 field; the others are
// derived from it (rows 0-1 only for the 12-real formats).  With naik set the
// operator is the improved one: weights c1 (one hop) and c3 (three hops), and
// the long links L_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu) in the same formats
// and layouts (ld18 ... lh12).
struct LinkSet {
    int fmt64;               // STAG_LINKS_F64_18 or STAG_LINKS_F64_12
    int fmt32;               // STAG_LINKS_F32_18 or STAG_LINKS_F16_12
    const double2* d18;
    const double2* d12;
    const float2* s18;
    const void* h12;         // __half2 [2][4][6][Vh]
    int naik;
    int nt;                  // FP64 links loaded non-temporally (fields larger than the Infinity Cache)
    double c1, c3;
    const double2* ld18;
    const double2* ld12;
    const float2* ls18;
    const void* lh12;
};

int dslash_grid(const Geom& g, int tps);

// FP64 operator (format fmt64)
void launch_dslash(const Geom& g, const LinkSet& ls, const double2* in, double2* out, int out_par, int tps,
                   const int* gate, hipStream_t s);
// out = c*in - D_eo w_o
void launch_dslash_axpy(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* in, double c,
                        double2* out, int tps, hipStream_t s);
// Ap = mt p - D_eo w_o and block partials of <p,Ap>, <r,Ap>, <Ap,Ap>
void launch_dslash_cg(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* p, const double2* r,
                      double2* Ap, const int* gate, double* dpart, int tps, hipStream_t s, double mass_term);
// res = b - (c x - D_eo w_o): block partials of |res|^2; res stored as float2 when r32_out != NULL
void launch_dslash_resid(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* x, const double2* b,
                         double c, double* part, int tps, hipStream_t s, float2* r32_out = nullptr);

template <class V>
struct FusedIterT;
// Iteration j of the fused multi-shift CG: step j-1's scalars and base update
// folded into w = D_oe p_j (first: j = 0, D_oe p_0 and |r_0|^2 partials only);
// always 4 threads per site, grid dslash_fused_grid(g) = dslash_grid(g, 4).
// double2: the FP64 operator (format fmt64); float2: FP32 Krylov vectors
// with the FP32 operator (format fmt32).
int dslash_fused_grid(const Geom& g);
void launch_dslash_fused(const Geom& g, const LinkSet& ls, const FusedIterT<double2>& f, double2* w_out, bool first,
                         hipStream_t s);
void launch_dslash_fused(const Geom& g, const LinkSet& ls, const FusedIterT<float2>& f, float2* w_out, bool first,
                         hipStream_t s);
// the D_eo launch of the fused loop: launch_dslash_cg with 4 threads per site
// and the operands' loads issued before the stop flag is tested
void launch_dslash_cg_fused(const Geom& g, const LinkSet& ls, const double2* w_o, const double2* p, const double2* r,
                            double2* Ap, const int* gate, double* dpart, hipStream_t s, double mass_term);
void launch_dslash_cg_fused(const Geom& g, const LinkSet& ls, const float2* w_o, const float2* p, const float2* r,
                            float2* Ap, const int* gate, double* dpart, hipStream_t s, double mass_term);

// FP32 operator (format fmt32)
void launch_dslash32(const Geom& g, const LinkSet& ls, const float2* in, float2* out, int out_par, int tps,
                     const int* gate, hipStream_t s);
void launch_dslash32_cg(const Geom& g, const LinkSet& ls, const float2* w_o, const float2* p, const float2* r,
                        float2* Ap, const int* gate, double* dpart, int tps, hipStream_t s, double mass_term);
void launch_dslash32_axpy(const Geom& g, const LinkSet& ls, const float2* w_o, const float2* in, double c,
                          float2* out, int tps, hipStream_t s);

// long links L_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu) (plain SU(3) products,
// no staggered signs) in the layout of the FP64 18-real links
void launch_long_links(const Geom& g, const double2* d18, double2* long18, hipStream_t s);
// link copies derived from an FP64 18-real field (the links or the long links)
void launch_links_to_d12(const Geom& g, const double2* d18, double2* d12, hipStream_t s);
void launch_links_to_s18(const Geom& g, const double2* d18, float2* s18, hipStream_t s);
void launch_links_to_h12(const Geom& g, const double2* d18, void* h12, hipStream_t s);

}  // namespace stag

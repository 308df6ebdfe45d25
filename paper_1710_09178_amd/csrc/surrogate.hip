// Learned force model: a gauge-covariant combination of the six plaquette
// staple forces of each link and of an optional auxiliary force field, with
// coefficients from an MLP (16 -> 64 -> 64 -> 8, SiLU) over gauge-invariant
// inputs (loop traces, parity and sign, the cosine of the auxiliary force
// with the staple sum).  Matrix products run on the
// bf16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation); everything
// else is FP32, the reductions of the loss and the gradients are fixed-order.
//
// Layout trick: every layer is computed transposed, Z^T = W * H^T, with the
// weights as the A operand and the activations (features x 16 links) as the
// B operand.  The 16x16 FP32 result of an MFMA (lane l holds rows
// 4*(l/16)+v, v<4, of column l%16) is then already in the B-operand layout of
// the next layer, so the forward pass needs no data movement between layers.
// Only the weight gradients (a sum over links, i.e. over the lane%16 index)
// go through an LDS transpose.
#include <cstring>
#include <vector>

#include "ctx.h"

namespace stag {

namespace {

constexpr int FI = 16, HD = 64, NO = 8, NCH = 7, NSTAPLE = 6;
// parameter offsets in one float array: W[out][in] row-major
constexpr int OW1 = 0, OB1 = OW1 + HD * FI, OW2 = OB1 + HD, OB2 = OW2 + HD * HD, OW3 = OB2 + HD,
              OB3 = OW3 + NO * HD, NPAR = OB3 + NO;
constexpr int kWavesSur = 4;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {  // round to nearest even
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}
// The LDS scratch of the tile loops is private to a wave and waves of a block
// may run different numbers of tiles, so ordering is per wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ __forceinline__ s4 pack4(float a, float b, float c, float d) {
    s4 r;
    r.x = (short)f2bf(a);
    r.y = (short)f2bf(b);
    r.z = (short)f2bf(c);
    r.w = (short)f2bf(d);
    return r;
}

// ---------------------------------------------------------------------------
// Features of every link (canonical link order n = 4 l + mu).
__device__ __forceinline__ M3 sload(const double2* __restrict__ links, const Geom& g, int x, int y, int z, int t,
                                    int mu) {
    const int par = (x + y + z + t) & 1;
    const int cb = cb_index(g, x, y, z, t);
    M3 m;
    const double2* u = links + link_off(g, par, mu, 0) + cb;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = u[(size_t)e * g.vh];
    return m;
}

__global__ __launch_bounds__(kBlock) void k_sur_features(Geom g, const double2* __restrict__ links,
                                                         const double* __restrict__ aux,
                                                         unsigned short* __restrict__ f, float* __restrict__ B) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = i / V, rem = i % V;
    const int par = rem / g.vh, cb = rem % g.vh;
    int c[4];
    cb_coords(g, par, cb, c[0], c[1], c[2], c[3]);
    const int n[4] = {g.nx, g.ny, g.nz, g.nt};
    const int l = c[0] + g.nx * (c[1] + g.ny * (c[2] + g.nz * c[3]));
    const size_t row = (size_t)4 * l + mu;
    const M3 U = sload(links, g, c[0], c[1], c[2], c[3], mu);
    float feat[FI];
#pragma unroll
    for (int k = 0; k < FI; ++k) feat[k] = 0.f;
    double gsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // sum of the staple forces
    int j = 0;
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int cp[4] = {c[0], c[1], c[2], c[3]};
        cp[mu] = (c[mu] + 1 == n[mu]) ? 0 : c[mu] + 1;
        int cn[4] = {c[0], c[1], c[2], c[3]};
        cn[nu] = (c[nu] + 1 == n[nu]) ? 0 : c[nu] + 1;
        int cm[4] = {c[0], c[1], c[2], c[3]};
        cm[nu] = (c[nu] == 0) ? n[nu] - 1 : c[nu] - 1;
        int cpm[4] = {cp[0], cp[1], cp[2], cp[3]};
        cpm[nu] = cm[nu];
        for (int ud = 0; ud < 2; ++ud) {
            M3 S;
            if (ud == 0) {
                const M3 a1 = sload(links, g, cp[0], cp[1], cp[2], cp[3], nu);
                const M3 a2 = sload(links, g, cn[0], cn[1], cn[2], cn[3], mu);
                const M3 a3 = sload(links, g, c[0], c[1], c[2], c[3], nu);
                S = m3_mul(m3_mul(a1, m3_dag(a2)), m3_dag(a3));
            } else {
                const M3 b1 = sload(links, g, cpm[0], cpm[1], cpm[2], cpm[3], nu);
                const M3 b2 = sload(links, g, cm[0], cm[1], cm[2], cm[3], mu);
                const M3 b3 = sload(links, g, cm[0], cm[1], cm[2], cm[3], nu);
                S = m3_mul(m3_mul(m3_dag(b1), m3_dag(b2)), b3);
            }
            const M3 L = m3_mul(U, S);
            const int ch = 2 * j + ud;
            feat[2 * ch] = (float)(L.e[0].x + L.e[4].x + L.e[8].x);
            feat[2 * ch + 1] = (float)(L.e[0].y + L.e[4].y + L.e[8].y);
            double b8[8];
            im_tr_ta(L, b8);
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                B[(row * NCH + ch) * 8 + a] = (float)b8[a];
                gsum[a] += b8[a];
            }
        }
        ++j;
    }
    feat[12] = par == 0 ? 1.f : -1.f;
    float sg = 1.f;
    if (mu == 1) sg = (c[0] & 1) ? -1.f : 1.f;
    if (mu == 2) sg = ((c[0] + c[1]) & 1) ? -1.f : 1.f;
    if (mu == 3) {
        sg = ((c[0] + c[1] + c[2]) & 1) ? -1.f : 1.f;
        if (c[3] == g.nt - 1) sg = -sg;
    }
    feat[13] = sg;
    // auxiliary channel and the cosine of its angle with the staple sum
    double ga[8], gg = 0.0, aa = 0.0, ag = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        ga[a] = aux ? aux[mom_off(g, par, mu, a) + cb] : 0.0;
        B[(row * NCH + NSTAPLE) * 8 + a] = (float)ga[a];
        gg += gsum[a] * gsum[a];
        aa += ga[a] * ga[a];
        ag += ga[a] * gsum[a];
    }
    feat[14] = aux ? (float)(ag / (sqrt(aa) * sqrt(gg) + 1e-30)) : 0.f;
#pragma unroll
    for (int k = 0; k < FI; ++k) f[row * FI + k] = f2bf(feat[k]);
}

// ---------------------------------------------------------------------------
// Weights staged in LDS as bf16, row-major [out][in].
struct WLds {
    unsigned short w1[HD * FI];
    unsigned short w2[HD * HD];
    unsigned short w3[16 * HD];  // rows 8..15 zero
    float b1[HD], b2[HD], b3[16];
};

__device__ void stage_weights(WLds& W, const float* __restrict__ prm) {
    for (int i = threadIdx.x; i < HD * FI; i += blockDim.x) W.w1[i] = f2bf(prm[OW1 + i]);
    for (int i = threadIdx.x; i < HD * HD; i += blockDim.x) W.w2[i] = f2bf(prm[OW2 + i]);
    for (int i = threadIdx.x; i < 16 * HD; i += blockDim.x) W.w3[i] = i < NO * HD ? f2bf(prm[OW3 + i]) : 0;
    for (int i = threadIdx.x; i < HD; i += blockDim.x) {
        W.b1[i] = prm[OB1 + i];
        W.b2[i] = prm[OB2 + i];
    }
    for (int i = threadIdx.x; i < 16; i += blockDim.x) W.b3[i] = i < NO ? prm[OB3 + i] : 0.f;
}

// A operand of rows [r0, r0+16) and columns [k0, k0+16) of a row-major bf16
// matrix with ld columns: lane l holds M[r0 + l%16][k0 + 4*(l/16) + v].
__device__ __forceinline__ s4 a_tile(const unsigned short* M, int ld, int r0, int k0) {
    const int l = threadIdx.x & 63;
    return *(const s4*)(M + (size_t)(r0 + (l & 15)) * ld + k0 + 4 * (l >> 4));
}
// A operand of the transposed matrix: lane l holds M[k0 + 4*(l/16)+v][r0 + l%16].
__device__ __forceinline__ s4 at_tile(const unsigned short* M, int ld, int r0, int k0) {
    const int l = threadIdx.x & 63;
    const int r = r0 + (l & 15), k = k0 + 4 * (l >> 4);
    s4 o;
    o.x = (short)M[(size_t)(k + 0) * ld + r];
    o.y = (short)M[(size_t)(k + 1) * ld + r];
    o.z = (short)M[(size_t)(k + 2) * ld + r];
    o.w = (short)M[(size_t)(k + 3) * ld + r];
    return o;
}

// Per-wave scratch for the transposes of one 16-link tile.
struct WaveLds {
    unsigned short h1T[HD * 16], h2T[HD * 16], dz2T[HD * 16], dz1T[HD * 16], fT[FI * 16], dcT[16 * 16];
    float c[16][NO];
    float dc[16][4][NO];
};

// Forward pass of one 16-link tile (rows n0..n0+15 of the dataset).  Returns
// the per-lane forward state; c (16 x 8) is left in W.c.
struct Fwd {
    f4 z1[4], z2[4];
    s4 h1b[4], h2b[4];
    s4 fb;
};

__device__ __forceinline__ void forward_tile(const WLds& W, WaveLds& S, const unsigned short* __restrict__ f, size_t n0,
                                             int nvalid, Fwd& F) {
    const int l = threadIdx.x & 63, col = l & 15, grp = l >> 4;
    if (col < nvalid)
        F.fb = *(const s4*)(f + (n0 + col) * FI + 4 * grp);
    else
        F.fb = s4{0, 0, 0, 0};
#pragma unroll
    for (int hb = 0; hb < 4; ++hb) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(a_tile(W.w1, FI, 16 * hb, 0), F.fb, acc);
        float h[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            F.z1[hb][v] = acc[v] + W.b1[16 * hb + 4 * grp + v];
            h[v] = silu_f(F.z1[hb][v]);
        }
        F.h1b[hb] = pack4(h[0], h[1], h[2], h[3]);
    }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma(a_tile(W.w2, HD, 16 * ob, 16 * kb), F.h1b[kb], acc);
        float h[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            F.z2[ob][v] = acc[v] + W.b2[16 * ob + 4 * grp + v];
            h[v] = silu_f(F.z2[ob][v]);
        }
        F.h2b[ob] = pack4(h[0], h[1], h[2], h[3]);
    }
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mfma(a_tile(W.w3, HD, 0, 16 * kb), F.h2b[kb], acc);
    if (grp < 2)
#pragma unroll
        for (int v = 0; v < 4; ++v) S.c[col][4 * grp + v] = acc[v] + W.b3[4 * grp + v];
}

// Loss, gradients and forces over a dataset slice.  One wave per 16-link tile
// (grid-stride); per-wave partial gradients go to gpart[wave][NPAR], partial
// losses to lpart[wave].  force_out: optional F (rows x 8).
__global__ __launch_bounds__(64 * kWavesSur) void k_sur_train(const unsigned short* __restrict__ f,
                                                              const float* __restrict__ B,
                                                              const float* __restrict__ target, long long rows,
                                                              double inv_rows, const float* __restrict__ prm,
                                                              float* __restrict__ gpart, double* __restrict__ lpart,
                                                              int want_grad) {
    __shared__ WLds W;
    __shared__ WaveLds SW[kWavesSur];
    stage_weights(W, prm);
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, col = l & 15, grp = l >> 4;
    WaveLds& S = SW[wave];
    const long long gw = (long long)blockIdx.x * kWavesSur + wave;
    const long long nw = (long long)gridDim.x * kWavesSur;
    f4 G2[4][4], G1[4], G3[4];
    float db1[4][4], db2[4][4], db3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        G1[a] = f4{0, 0, 0, 0};
        G3[a] = f4{0, 0, 0, 0};
        db3[a] = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            G2[a][b] = f4{0, 0, 0, 0};
            db1[a][b] = db2[a][b] = 0.f;
        }
    }
    double loss = 0.0;
    const long long ntiles = (rows + 15) / 16;
    for (long long tile = gw; tile < ntiles; tile += nw) {
        const size_t n0 = (size_t)tile * 16;
        const int nvalid = (int)(rows - (long long)n0 < 16 ? rows - (long long)n0 : 16);
        Fwd F;
        forward_tile(W, S, f, n0, nvalid, F);
        wave_sync();
        // force, loss and dL/dc: lane (col, grp) handles components a = 2 grp, 2 grp + 1
        float dcp[NO];
#pragma unroll
        for (int j = 0; j < NO; ++j) dcp[j] = 0.f;
        if (col < nvalid) {
            const size_t n = n0 + col;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int a = 2 * grp + q;
                float Fa = 0.f;
#pragma unroll
                for (int j = 0; j < NCH; ++j) Fa += S.c[col][j] * B[(n * NCH + j) * 8 + a];
                const float d = Fa - target[n * 8 + a];
                loss += (double)d * (double)d;
                const float dF = (float)(2.0 * inv_rows) * d;
#pragma unroll
                for (int j = 0; j < NCH; ++j) dcp[j] += dF * B[(n * NCH + j) * 8 + a];
            }
        }
        if (!want_grad) {
            wave_sync();
            continue;
        }
#pragma unroll
        for (int j = 0; j < NO; ++j) S.dc[col][grp][j] = dcp[j];
        wave_sync();
        // dC^T as a B operand: lane holds dc[n = col][j = 4 grp + v] (j < 8)
        float dcv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = 4 * grp + v;
            dcv[v] = (grp < 2) ? S.dc[col][0][j] + S.dc[col][1][j] + S.dc[col][2][j] + S.dc[col][3][j] : 0.f;
        }
        const s4 dcb = pack4(dcv[0], dcv[1], dcv[2], dcv[3]);
#pragma unroll
        for (int v = 0; v < 4; ++v) db3[v] += dcv[v];
        // dH2^T = W3^T dC^T, dZ2 = dH2 * silu'(z2)
        s4 dz2b[4];
        float dz2[4][4];
#pragma unroll
        for (int hb = 0; hb < 4; ++hb) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(at_tile(W.w3, HD, 16 * hb, 0), dcb, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) dz2[hb][v] = acc[v] * dsilu_f(F.z2[hb][v]);
            dz2b[hb] = pack4(dz2[hb][0], dz2[hb][1], dz2[hb][2], dz2[hb][3]);
#pragma unroll
            for (int v = 0; v < 4; ++v) db2[hb][v] += dz2[hb][v];
        }
        // dH1^T = W2^T dZ2^T, dZ1 = dH1 * silu'(z1)
        s4 dz1b[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = mfma(at_tile(W.w2, HD, 16 * ib, 16 * kb), dz2b[kb], acc);
            float dz1[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                dz1[v] = acc[v] * dsilu_f(F.z1[ib][v]);
                db1[ib][v] += dz1[v];
            }
            dz1b[ib] = pack4(dz1[0], dz1[1], dz1[2], dz1[3]);
        }
        // weight gradients: transpose activations and deltas through LDS as
        // [feature][link] so that 4 consecutive links are one 8-byte read
#pragma unroll
        for (int hb = 0; hb < 4; ++hb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int h = 16 * hb + 4 * grp + v;
                S.h1T[h * 16 + col] = (unsigned short)F.h1b[hb][v];
                S.h2T[h * 16 + col] = (unsigned short)F.h2b[hb][v];
                S.dz2T[h * 16 + col] = (unsigned short)dz2b[hb][v];
                S.dz1T[h * 16 + col] = (unsigned short)dz1b[hb][v];
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            S.fT[(4 * grp + v) * 16 + col] = (unsigned short)F.fb[v];
            S.dcT[(4 * grp + v) * 16 + col] = (unsigned short)dcb[v];
        }
        wave_sync();
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            const s4 a2 = a_tile(S.dz2T, 16, 16 * ob, 0);
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) G2[ob][ib] = mfma(a2, a_tile(S.h1T, 16, 16 * ib, 0), G2[ob][ib]);
            G1[ob] = mfma(a_tile(S.dz1T, 16, 16 * ob, 0), a_tile(S.fT, 16, 0, 0), G1[ob]);
            G3[ob] = mfma(a_tile(S.dcT, 16, 0, 0), a_tile(S.h2T, 16, 16 * ob, 0), G3[ob]);
        }
        wave_sync();
    }
    // per-wave partials (fixed order: wave index)
    if (want_grad) {
        float* out = gpart + (size_t)gw * NPAR;
        // G tiles: lane holds rows 4 grp + v of column col
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * ob + 4 * grp + v;
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) out[OW2 + o * HD + 16 * ib + col] = G2[ob][ib][v];
                out[OW1 + o * FI + col] = G1[ob][v];
                if (4 * grp + v < NO) out[OW3 + (4 * grp + v) * HD + 16 * ob + col] = G3[ob][v];
            }
        // bias sums: reduce the 16 links (cols) held by the lanes of a group
#pragma unroll
        for (int hb = 0; hb < 4; ++hb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float s1 = db1[hb][v], s2 = db2[hb][v];
#pragma unroll
                for (int off = 8; off >= 1; off >>= 1) {
                    s1 += __shfl_xor(s1, off, 16);
                    s2 += __shfl_xor(s2, off, 16);
                }
                if (col == 0) {
                    out[OB1 + 16 * hb + 4 * grp + v] = s1;
                    out[OB2 + 16 * hb + 4 * grp + v] = s2;
                }
            }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float s3 = db3[v];
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) s3 += __shfl_xor(s3, off, 16);
            if (col == 0 && 4 * grp + v < NO) out[OB3 + 4 * grp + v] = s3;
        }
    }
    // loss partial of the wave
    double lw = loss;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) lw += __shfl_xor(lw, off, 64);
    if (l == 0) lpart[gw] = lw;
}

// Forces F = sum_j c_j B_j of the current gauge field, written (dt == 0) or
// added (dt != 0, times dt) to the internal momentum layout.
__global__ __launch_bounds__(64 * kWavesSur) void k_sur_apply(Geom g, const unsigned short* __restrict__ f,
                                                              const float* __restrict__ B, const float* __restrict__ prm,
                                                              double* __restrict__ mom, double dt) {
    __shared__ WLds W;
    __shared__ WaveLds SW[kWavesSur];
    stage_weights(W, prm);
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, col = l & 15, grp = l >> 4;
    WaveLds& S = SW[wave];
    const long long rows = 8LL * g.vh;
    const long long ntiles = (rows + 15) / 16;
    const long long gw = (long long)blockIdx.x * kWavesSur + wave;
    const long long nw = (long long)gridDim.x * kWavesSur;
    for (long long tile = gw; tile < ntiles; tile += nw) {
        const size_t n0 = (size_t)tile * 16;
        const int nvalid = (int)(rows - (long long)n0 < 16 ? rows - (long long)n0 : 16);
        Fwd F;
        forward_tile(W, S, f, n0, nvalid, F);
        wave_sync();
        if (col < nvalid) {
            const size_t n = n0 + col;
            const int lsite = (int)(n >> 2), mu = (int)(n & 3);
            const int x = lsite % g.nx, r1 = lsite / g.nx;
            const int y = r1 % g.ny, r2 = r1 / g.ny;
            const int z = r2 % g.nz, t = r2 / g.nz;
            const int par = (x + y + z + t) & 1, cb = lsite >> 1;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int a = 2 * grp + q;
                float Fa = 0.f;
#pragma unroll
                for (int j = 0; j < NCH; ++j) Fa += S.c[col][j] * B[(n * NCH + j) * 8 + a];
                double* m = mom + mom_off(g, par, mu, a) + cb;
                if (dt == 0.0)
                    *m = (double)Fa;
                else
                    *m += dt * (double)Fa;
            }
        }
        wave_sync();
    }
}

// Targets in dataset order (canonical links, 8 floats each) from a force field
// in the internal momentum layout.
__global__ void k_sur_target(Geom g, const double* __restrict__ force, float* __restrict__ tgt) {
    const int V = 2 * g.vh;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = i / V, rem = i % V;
    const int par = rem / g.vh, cb = rem % g.vh;
    int x, y, z, t;
    cb_coords(g, par, cb, x, y, z, t);
    const size_t row = (size_t)4 * (x + g.nx * (y + g.ny * (z + g.nz * t))) + mu;
#pragma unroll
    for (int a = 0; a < 8; ++a) tgt[row * 8 + a] = (float)force[mom_off(g, par, mu, a) + cb];
}

// Sum of per-wave partial gradients (wave order) and one Adam step
// (Kingma & Ba 2015, bias-corrected) on the FP32 master parameters.
// Gradient sum, first stage: chunk c (blockIdx.y) of the per-wave partials,
// waves in order, one thread per parameter.
constexpr int kGradChunks = 32;
__global__ void k_sur_gsum(const float* __restrict__ gpart, int nwaves, float* __restrict__ gpart2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPAR) return;
    const int per = (nwaves + kGradChunks - 1) / kGradChunks;
    const int w0 = blockIdx.y * per, w1 = min(nwaves, w0 + per);
    float g = 0.f;
    for (int w = w0; w < w1; ++w) g += gpart[(size_t)w * NPAR + k];
    gpart2[(size_t)blockIdx.y * NPAR + k] = g;
}

// Second stage (chunks in order) and one Adam step.
__global__ void k_sur_adam(const float* __restrict__ gpart2, float* __restrict__ prm, float* __restrict__ m,
                           float* __restrict__ v, float* __restrict__ grad_out, float lr, float b1, float b2, float eps,
                           float c1, float c2, int step) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPAR) return;
    float gsum = 0.f;
    for (int c = 0; c < kGradChunks; ++c) gsum += gpart2[(size_t)c * NPAR + k];
    if (grad_out) grad_out[k] = gsum;
    if (!step) return;
    const float mk = b1 * m[k] + (1.f - b1) * gsum;
    const float vk = b2 * v[k] + (1.f - b2) * gsum * gsum;
    m[k] = mk;
    v[k] = vk;
    prm[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// out[0] = sum of the n partials (one block, fixed order); out[1] += the same
// sum (epoch accumulator), or out[1] = 0 first when reset is set
__global__ __launch_bounds__(kBlock) void k_sum_double(const double* __restrict__ p, int n, double* __restrict__ out,
                                                       int reset) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += kBlock) v[0] += p[i];
    __shared__ double lds[4];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = (reset ? 0.0 : out[1]) + v[0];
    }
}

}  // namespace
}  // namespace stag

using namespace stag;

struct stag_surrogate {
    stag_ctx* lat = nullptr;
    int capacity = 0, pairs = 0;
    long long links = 0;               // links per configuration
    unsigned short* f = nullptr;       // [capacity+1][links][16] bf16 (slot `capacity` = scratch)
    float* B = nullptr;                // [capacity+1][links][6][8]
    float* tgt = nullptr;              // [capacity+1][links][8]
    float* prm = nullptr;              // [NPAR] FP32 master parameters
    float* m = nullptr;
    float* v = nullptr;
    float* gpart = nullptr;            // [nwaves][NPAR]
    float* gpart2 = nullptr;           // [kGradChunks][NPAR]
    const double* aux = nullptr;       // auxiliary force field (internal momentum layout) or NULL
    float* grad = nullptr;             // [NPAR]
    double* lpart = nullptr;
    double* lsum = nullptr;
    double* lsum_host = nullptr;
    int nblocks = 0;
    int adam_t = 0;
    std::string err;
};

namespace {

stag_status sfail(stag_surrogate* s, stag_status code, const std::string& m) {
    if (s) s->err = m;
    return code;
}

#define SHIP(s, expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return sfail((s), STAG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
stag_status salloc(stag_surrogate* s, T** p, size_t bytes) {
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return sfail(s, STAG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return STAG_OK;
}

unsigned short* slot_f(stag_surrogate* s, int k) { return s->f + (size_t)k * s->links * FI; }
float* slot_B(stag_surrogate* s, int k) { return s->B + (size_t)k * s->links * NCH * 8; }
float* slot_t(stag_surrogate* s, int k) { return s->tgt + (size_t)k * s->links * 8; }

void features_into(stag_surrogate* s, int k) {
    stag_ctx* c = s->lat;
    const int grid = (int)((s->links + kBlock - 1) / kBlock);
    k_sur_features<<<grid, kBlock, 0, c->s>>>(c->g, c->links, s->aux, slot_f(s, k), slot_B(s, k));
}

// loss (and gradient sum / Adam step) over `rows` dataset rows starting at slot k
void train_pass(stag_surrogate* s, int k, long long rows, bool grad, int adam_step, float lr, bool reset = true) {
    stag_ctx* c = s->lat;
    k_sur_train<<<s->nblocks, 64 * kWavesSur, 0, c->s>>>(slot_f(s, k), slot_B(s, k), slot_t(s, k), rows,
                                                         1.0 / (double)rows, s->prm, s->gpart, s->lpart, grad ? 1 : 0);
    if (grad) {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = adam_step ? 1.f - powf(b1, (float)adam_step) : 1.f;
        const float c2 = adam_step ? 1.f - powf(b2, (float)adam_step) : 1.f;
        k_sur_gsum<<<dim3((NPAR + 255) / 256, kGradChunks), 256, 0, c->s>>>(s->gpart, s->nblocks * kWavesSur,
                                                                             s->gpart2);
        k_sur_adam<<<(NPAR + 255) / 256, 256, 0, c->s>>>(s->gpart2, s->prm, s->m, s->v, s->grad, lr, b1, b2, 1e-8f, c1,
                                                         c2, adam_step);
    }
    k_sum_double<<<1, kBlock, 0, c->s>>>(s->lpart, s->nblocks * kWavesSur, s->lsum, reset ? 1 : 0);
}

}  // namespace

extern "C" {

stag_status stag_surrogate_create(stag_surrogate_handle* out, stag_handle lat, int capacity, uint64_t seed) {
    if (!out || !lat || capacity < 0) return STAG_ERR_INVALID_ARG;
    *out = nullptr;
    stag_surrogate* s = new stag_surrogate();
    s->lat = lat;
    s->capacity = capacity;
    s->links = 8LL * lat->g.vh;
    s->nblocks = 256;
    const size_t slots = (size_t)capacity + 1;
    stag_status e;
    if ((e = salloc(s, &s->f, slots * s->links * FI * 2)) || (e = salloc(s, &s->B, slots * s->links * NCH * 8 * 4)) ||
        (e = salloc(s, &s->tgt, slots * s->links * 8 * 4)) || (e = salloc(s, &s->prm, NPAR * 4)) ||
        (e = salloc(s, &s->m, NPAR * 4)) || (e = salloc(s, &s->v, NPAR * 4)) ||
        (e = salloc(s, &s->gpart, (size_t)s->nblocks * kWavesSur * NPAR * 4)) ||
        (e = salloc(s, &s->gpart2, (size_t)kGradChunks * NPAR * 4)) || (e = salloc(s, &s->grad, NPAR * 4)) ||
        (e = salloc(s, &s->lpart, (size_t)s->nblocks * kWavesSur * 8)) || (e = salloc(s, &s->lsum, 16))) {
        lat->err = s->err;
        stag_surrogate_destroy(s);
        return e;
    }
    if (hipHostMalloc((void**)&s->lsum_host, 16, hipHostMallocDefault) != hipSuccess) {
        stag_surrogate_destroy(s);
        return STAG_ERR_OOM;
    }
    // He-style initial parameters from a seeded host generator (last layer small)
    std::vector<float> p(NPAR, 0.f);
    uint64_t st = seed * 0x9E3779B97F4A7C15ULL + 1;
    auto uni = [&]() {
        st ^= st >> 12;
        st ^= st << 25;
        st ^= st >> 27;
        return ((st * 0x2545F4914F6CDD1DULL) >> 11) * (1.0 / 9007199254740992.0);
    };
    auto gauss = [&]() { return std::sqrt(-2.0 * std::log(uni() + 1e-300)) * std::cos(6.283185307179586 * uni()); };
    for (int i = 0; i < HD * FI; ++i) p[OW1 + i] = (float)(gauss() * std::sqrt(2.0 / FI));
    for (int i = 0; i < HD * HD; ++i) p[OW2 + i] = (float)(gauss() * std::sqrt(2.0 / HD));
    for (int i = 0; i < NO * HD; ++i) p[OW3 + i] = (float)(gauss() * 0.01);
    hipMemcpy(s->prm, p.data(), NPAR * 4, hipMemcpyHostToDevice);
    hipMemset(s->m, 0, NPAR * 4);
    hipMemset(s->v, 0, NPAR * 4);
    *out = s;
    return STAG_OK;
}

stag_status stag_surrogate_destroy(stag_surrogate_handle s) {
    if (!s) return STAG_OK;
    if (s->lat && s->lat->s) hipStreamSynchronize(s->lat->s);
    void* bufs[] = {s->f, s->B, s->tgt, s->prm, s->m, s->v, s->gpart, s->gpart2, s->grad, s->lpart, s->lsum};
    for (void* b : bufs)
        if (b) hipFree(b);
    if (s->lsum_host) hipHostFree(s->lsum_host);
    delete s;
    return STAG_OK;
}

const char* stag_surrogate_last_error(stag_surrogate_handle s) { return s ? s->err.c_str() : ""; }

int stag_surrogate_param_count(void) { return NPAR; }

stag_status stag_surrogate_params(stag_surrogate_handle s, float* get_out, const float* set_in) {
    if (!s) return STAG_ERR_INVALID_ARG;
    if (set_in) {
        SHIP(s, hipMemcpy(s->prm, set_in, NPAR * 4, hipMemcpyHostToDevice));
        SHIP(s, hipMemset(s->m, 0, NPAR * 4));
        SHIP(s, hipMemset(s->v, 0, NPAR * 4));
        s->adam_t = 0;
    }
    if (get_out) SHIP(s, hipMemcpy(get_out, s->prm, NPAR * 4, hipMemcpyDeviceToHost));
    return STAG_OK;
}

stag_status stag_surrogate_set_aux(stag_surrogate_handle s, const void* aux) {
    if (!s || (uintptr_t)aux % 16) return sfail(s, STAG_ERR_INVALID_ARG, "bad arguments");
    s->aux = (const double*)aux;
    return STAG_OK;
}

int stag_surrogate_pair_count(stag_surrogate_handle s) { return s ? s->pairs : 0; }

int stag_surrogate_capacity(stag_surrogate_handle s) { return s ? s->capacity : 0; }

stag_status stag_surrogate_add_pair(stag_surrogate_handle s, const void* force) {
    if (!s || !force || (uintptr_t)force % 16) return sfail(s, STAG_ERR_INVALID_ARG, "bad arguments");
    if (s->pairs >= s->capacity) return sfail(s, STAG_ERR_INVALID_ARG, "dataset is full");
    stag_ctx* c = s->lat;
    if (!c->has_gauge) return sfail(s, STAG_ERR_NO_GAUGE, "lattice has no gauge field");
    features_into(s, s->pairs);
    k_sur_target<<<(int)((s->links + 255) / 256), 256, 0, c->s>>>(c->g, (const double*)force, slot_t(s, s->pairs));
    SHIP(s, hipGetLastError());
    SHIP(s, hipStreamSynchronize(c->s));
    s->pairs += 1;
    return STAG_OK;
}

stag_status stag_surrogate_train(stag_surrogate_handle s, int epochs, double lr, double* loss_out) {
    if (!s || epochs < 0 || !(lr > 0)) return sfail(s, STAG_ERR_INVALID_ARG, "bad arguments");
    if (s->pairs == 0) return sfail(s, STAG_ERR_INVALID_ARG, "no training pairs");
    double last = 0.0;
    for (int ep = 0; ep < epochs; ++ep) {
        // one Adam step per stored configuration; the loss is summed on the
        // device and read once per epoch
        for (int k = 0; k < s->pairs; ++k) {
            s->adam_t += 1;
            train_pass(s, k, s->links, true, s->adam_t, (float)lr, k == 0);
        }
        SHIP(s, hipMemcpyAsync(s->lsum_host, s->lsum, 16, hipMemcpyDeviceToHost, s->lat->s));
        SHIP(s, hipStreamSynchronize(s->lat->s));
        last = s->lsum_host[1] / (double)s->links / s->pairs;
    }
    if (loss_out) *loss_out = last;
    SHIP(s, hipGetLastError());
    return STAG_OK;
}

stag_status stag_surrogate_eval(stag_surrogate_handle s, const void* force, double* loss_out, float* grad_out) {
    if (!s || !force || (uintptr_t)force % 16) return sfail(s, STAG_ERR_INVALID_ARG, "bad arguments");
    stag_ctx* c = s->lat;
    if (!c->has_gauge) return sfail(s, STAG_ERR_NO_GAUGE, "lattice has no gauge field");
    const int k = s->capacity;  // scratch slot
    features_into(s, k);
    k_sur_target<<<(int)((s->links + 255) / 256), 256, 0, c->s>>>(c->g, (const double*)force, slot_t(s, k));
    train_pass(s, k, s->links, grad_out != nullptr, 0, 0.f);
    SHIP(s, hipMemcpyAsync(s->lsum_host, s->lsum, 8, hipMemcpyDeviceToHost, c->s));
    if (grad_out) SHIP(s, hipMemcpyAsync(grad_out, s->grad, NPAR * 4, hipMemcpyDeviceToHost, c->s));
    SHIP(s, hipStreamSynchronize(c->s));
    if (loss_out) *loss_out = s->lsum_host[0] / (double)s->links;
    return STAG_OK;
}

stag_status stag_surrogate_force(stag_surrogate_handle s, void* mom, double dt) {
    if (!s || !mom || (uintptr_t)mom % 16) return sfail(s, STAG_ERR_INVALID_ARG, "bad arguments");
    stag_ctx* c = s->lat;
    if (!c->has_gauge) return sfail(s, STAG_ERR_NO_GAUGE, "lattice has no gauge field");
    const int k = s->capacity;
    features_into(s, k);
    k_sur_apply<<<s->nblocks, 64 * kWavesSur, 0, c->s>>>(c->g, slot_f(s, k), slot_B(s, k), s->prm, (double*)mom, dt);
    SHIP(s, hipGetLastError());
    return STAG_OK;
}

}  // extern "C"

// HIP kernels of the forward 3DGS rasterizer for CDNA4 (gfx950, wave64).
//
//   k_preprocess   per Gaussian (x views): activation, 3D covariance, camera
//                  transform, projection, EWA 2D covariance + conic (FP64
//                  fallback when near-singular), SH colour, screen footprint
//   k_chunk_totals, k_scan_*
//                  exclusive scans of per-block counts (chunk totals, then
//                  each chunk; wave64 DPP scans)
//   k_compact      visible Gaussians as (depth key, record, packed tile
//                  rectangle) triples; the FP64 conics of the near-singular
//                  Gaussians
//   k_sort_*       LSD radix sort passes, 8-bit digits, reduce-then-scan,
//                  LDS-atomic digit counts, ballot/mbcnt ranking inside a
//                  wave, DPP scans; the depth digits of the (tile | depth)
//                  keys are sorted on the visible Gaussians before
//                  duplication, the tile digits on the duplicates after it
//   k_sorted_sums  tile counts per 256 depth-ordered Gaussians
//   k_duplicate    one (tile | depth) key per (Gaussian, overlapped tile)
//   k_duplicate_culled
//                  the same, keeping only the tiles where the Gaussian can
//                  reach the skip threshold at some pixel (count, then emit)
//   k_ranges       [start, end) of every tile in the sorted list
//   k_bin_*        single views: the tile digit placed by counting instead
//                  (per-block tile histograms from 2D difference grids, their
//                  prefixes, then every (Gaussian, tile) entry written straight
//                  to its sorted position; the ranges are the tile starts)
//   k_blend        front-to-back compositing, one wave64 per 8x8 pixel block,
//                  Gaussians staged per wave in LDS, per-wave early exit
//
// Numerics: all kernels are compiled with -ffp-contract=off; every fused
// multiply-add is written explicitly so the FP32 operation sequence is fixed.
#include "tigas_internal.h"

namespace tigas {

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ uint32_t bits_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP row shifts and
// row broadcasts (all 64 lanes must be active).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return readlane(wave_incl_scan(v), 63); }

// Inclusive prefix maximum over the 64 lanes of a wave (same lane pattern as
// wave_incl_scan; lanes without a source see 0, the identity for unsigned
// maxima).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// Exclusive scan over a workgroup of NT threads; *total receives the sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
    const uint32_t incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) lds[w] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const uint32_t s = lds[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    *total = tot;
    __syncthreads();
    return off + incl - v;
}

template <int NT>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* lds) {
    uint32_t tot;
    block_excl_scan<NT>(v, lds, &tot);
    return tot;
}

// ------------------------------------------------------ double-float helpers
// Error-free transformations (Knuth two-sum, fma two-product) so that the
// pixel position of a Gaussian is carried as an unevaluated FP32 sum hi + lo.

struct df {
    float hi, lo;
};
__device__ __forceinline__ df two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ df quick_two_sum(float a, float b) {
    const float s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ df df_add(df a, df b) {
    df s = two_sum(a.hi, b.hi);
    s.lo = s.lo + (a.lo + b.lo);
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ df df_mulf(df a, float b) {
    const float p = a.hi * b;
    float e = __builtin_fmaf(a.hi, b, -p);
    e = __builtin_fmaf(a.lo, b, e);
    return quick_two_sum(p, e);
}
__device__ __forceinline__ df df_div(df a, df b) {
    const float q1 = a.hi / b.hi;
    const df p = df_mulf(b, q1);
    const df r = df_add(a, df{-p.hi, -p.lo});
    const float q2 = r.hi / b.hi;
    return quick_two_sum(q1, q2);
}

// --------------------------------------------------------- attribute decode

__device__ __forceinline__ float h2f(uint32_t bits16, int storage) {
    if (storage == 2) return __uint_as_float(bits16 << 16);  // bfloat16
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}
__device__ __forceinline__ void unpack8(const uint4 u, float* f, int storage) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = h2f(w[i] & 0xffffu, storage);
        f[2 * i + 1] = h2f(w[i] >> 16, storage);
    }
}

// Real spherical harmonics with the Condon-Shortley phase, degree <= 3
// (textbook normalisations), colour = 0.5 + sum Y_i k_i, clamped below at 0.
constexpr float SH_C0 = 0.28209479177387814f;
constexpr float SH_C1 = 0.48860251190291992f;
constexpr float SH_C2A = 1.0925484305920792f;
constexpr float SH_C2B = 0.31539156525252005f;
constexpr float SH_C2C = 0.54627421529603959f;
constexpr float SH_C3A = 0.59004358992664352f;
constexpr float SH_C3B = 2.8906114426405538f;
constexpr float SH_C3C = 0.45704579946446577f;
constexpr float SH_C3D = 0.3731763325901154f;
constexpr float SH_C3E = 1.4453057213202769f;

template <int DEG>
__device__ __forceinline__ void sh_colour(const float* k, float x, float y, float z, int deg, float* rgb) {
    float Y[16];
    Y[0] = SH_C0;
    if (DEG >= 1) {
        Y[1] = -SH_C1 * y;
        Y[2] = SH_C1 * z;
        Y[3] = -SH_C1 * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = SH_C2A * (x * y);
        Y[5] = -SH_C2A * (y * z);
        Y[6] = SH_C2B * (3.0f * zz - 1.0f);
        Y[7] = -SH_C2A * (x * z);
        Y[8] = SH_C2C * (xx - yy);
        if (DEG >= 3) {
            Y[9] = -SH_C3A * (y * (3.0f * xx - yy));
            Y[10] = SH_C3B * (x * y * z);
            Y[11] = -SH_C3C * (y * (5.0f * zz - 1.0f));
            Y[12] = SH_C3D * (z * (5.0f * zz - 3.0f));
            Y[13] = -SH_C3C * (x * (5.0f * zz - 1.0f));
            Y[14] = SH_C3E * (z * (xx - yy));
            Y[15] = -SH_C3A * (x * (xx - 3.0f * yy));
        }
    }
    const int nc = (DEG + 1) * (DEG + 1);
    const int nuse = (deg + 1) * (deg + 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float s = 0.5f;
#pragma unroll
        for (int i = 0; i < nc; ++i)
            if (i < nuse) s = __builtin_fmaf(Y[i], k[i * 3 + ch], s);
        rgb[ch] = fmaxf(s, 0.0f);
    }
}

// ------------------------------------------------------------- preprocess

constexpr float NEAR_Z = 0.2f;
constexpr float DILATION = 0.3f;
constexpr float ALPHA_MIN = 1.0f / 255.0f;
// log2(1/255): below it, 2^e < 1/255 and a Gaussian is skipped at the pixel.
constexpr float LOG2_ALPHA_MIN = -7.99435343685886f;
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN255 = 5.5412635451584258f;
constexpr float KAPPA_INV = 1.0f / 64.0f;  // FP64 fallback when a*c > 64 det

// FP64 recomputation of the 2D covariance from the FP32 inputs.
__device__ __forceinline__ void cov2d_fp64(const float* q32, const float* ls32, float mx, float my, float mz,
                                        const ViewParams& v, double* abc) {
    double qw = q32[0], qx = q32[1], qy = q32[2], qz = q32[3];
    const double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                         2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                         2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    const double s[3] = {exp((double)ls32[0]), exp((double)ls32[1]), exp((double)ls32[2])};
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] * s[j];
    const double d[3] = {(double)mx - (double)v.cam[0], (double)my - (double)v.cam[1], (double)mz - (double)v.cam[2]};
    double p[3];
    for (int i = 0; i < 3; ++i)
        p[i] = (double)v.V[i * 3] * d[0] + (double)v.V[i * 3 + 1] * d[1] + (double)v.V[i * 3 + 2] * d[2];
    double rx = p[0] / p[2], ry = p[1] / p[2];
    rx = fmin(fmax(rx, -(double)v.lim_x), (double)v.lim_x);
    ry = fmin(fmax(ry, -(double)v.lim_y), (double)v.lim_y);
    const double fxz = (double)v.fx / p[2], fyz = (double)v.fy / p[2];
    double T0[3], T1[3];
    for (int j = 0; j < 3; ++j) {
        T0[j] = fxz * ((double)v.V[j] - rx * (double)v.V[6 + j]);
        T1[j] = fyz * ((double)v.V[3 + j] - ry * (double)v.V[6 + j]);
    }
    double m0[3], m1[3];
    for (int k = 0; k < 3; ++k) {
        m0[k] = T0[0] * M[k] + T0[1] * M[3 + k] + T0[2] * M[6 + k];
        m1[k] = T1[0] * M[k] + T1[1] * M[3 + k] + T1[2] * M[6 + k];
    }
    abc[0] = m0[0] * m0[0] + m0[1] * m0[1] + m0[2] * m0[2] + (double)DILATION;
    abc[1] = m0[0] * m1[0] + m0[1] * m1[1] + m0[2] * m1[2];
    abc[2] = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2] + (double)DILATION;
}

// SH coefficients of Gaussian g (the words of degree <= DEG) decoded to FP32.
template <int ST, int DEG>
__device__ __forceinline__ void load_sh(const SceneView& s, int64_t n, int64_t g, float* k) {
    if (ST == 0) {
        const float4* sh = reinterpret_cast<const float4*>(s.sh);
        constexpr int NP = ((DEG + 1) * (DEG + 1) * 3 + 3) / 4;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const float4 t = sh[g * s.sh_stride + p];
            k[4 * p] = t.x;
            k[4 * p + 1] = t.y;
            k[4 * p + 2] = t.z;
            k[4 * p + 3] = t.w;
        }
    } else {
        const uint4* sh = reinterpret_cast<const uint4*>(s.sh);
        constexpr int NP = ((DEG + 1) * (DEG + 1) * 3 + 7) / 8;
#pragma unroll
        for (int p = 0; p < NP; ++p) unpack8(sh[g * s.sh_stride + p], &k[8 * p], ST);
    }
}

// Bit d set when the SH coefficients of degrees 0..d are all finite.
__host__ __device__ constexpr int sh_degree_of(int i) {  // float i of the [16][3] coefficient block
    return i < 3 ? 0 : i < 12 ? 1 : i < 27 ? 2 : 3;
}
template <int DEG>
__device__ __forceinline__ uint32_t sh_finite(const float* k) {
    uint32_t bad = 0;  // bit d: a coefficient of degree d is not finite
#pragma unroll
    for (int i = 0; i < 3 * (DEG + 1) * (DEG + 1); ++i)
        bad |= __builtin_isfinite(k[i]) ? 0u : (1u << sh_degree_of(i));
    // lowest bad degree b: degrees below b are fine
    return (bad & (0u - bad)) - 1u;
}

template <int ST, int DEG>
__global__ __launch_bounds__(K1_THREADS) void k_preprocess(SceneView s, const ViewParams* __restrict__ views,
                                                           int nviews, uint32_t rec_base, uint32_t n_pad,
                                                           uint32_t view_base, PreOut o) {
    __shared__ uint32_t red[2][K1_THREADS / 64][3];
    const int64_t g = (int64_t)blockIdx.x * K1_THREADS + threadIdx.x;
    const bool in = g < s.n;
    const int64_t n = s.n;

    // ---- view-independent attributes
    float mx = 0.f, my = 0.f, mz = 0.f;
    float q[4] = {1.f, 0.f, 0.f, 0.f}, ls[3] = {0.f, 0.f, 0.f}, logit = 0.f;
    if (in) {
        mx = s.mean[g];
        my = s.mean[n + g];
        mz = s.mean[2 * n + g];
        if (ST == 0) {
            const float4* a = reinterpret_cast<const float4*>(s.attr);
            const float4 r = a[g], m = a[n + g];
            q[0] = r.x; q[1] = r.y; q[2] = r.z; q[3] = r.w;
            ls[0] = m.x; ls[1] = m.y; ls[2] = m.z; logit = m.w;
        } else {
            float f[8];
            unpack8(reinterpret_cast<const uint4*>(s.attr)[g], f, ST);
            q[0] = f[0]; q[1] = f[1]; q[2] = f[2]; q[3] = f[3];
            ls[0] = f[4]; ls[1] = f[5]; ls[2] = f[6]; logit = f[7];
        }
    }
    const float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    bool ok = in && qn2 > 0.0f && __builtin_isfinite(qn2) && __builtin_isfinite(mx) && __builtin_isfinite(my) &&
              __builtin_isfinite(mz) && __builtin_isfinite(ls[0]) && __builtin_isfinite(ls[1]) &&
              __builtin_isfinite(ls[2]) && __builtin_isfinite(logit);
    // opacity and its log2 (folded into the blend exponent)
    const float op = 1.0f / (1.0f + expf(-logit));
    ok = ok && op >= ALPHA_MIN;
    const float L = log2f(op);
    // alpha >= 1/255 support: Q <= 2 ln(255 o); widened by 2^-9 relative and
    // 2^-12 absolute so FP32 evaluation error cannot push a contributing
    // pixel outside the footprint
    const float k2 = 2.0f * __builtin_fmaf(L, 0.69314718055994531f, LN255);
    const float k2m = __builtin_fmaf(k2, 1.0f + 1.0f / 512.0f, 1.0f / 4096.0f);
    // M = Rq diag(exp(ls)), Sigma = M M^T
    float M[9];
    float smax = 0.0f;  // largest scale: bounds the screen footprint before the EWA step
    {
        const float inv = 1.0f / sqrtf(qn2);
        const float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
        const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                            2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                            2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
        const float sc[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
        smax = fmaxf(sc[0], fmaxf(sc[1], sc[2]));
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] * sc[j];
    }

    float k[48];
    bool sh_loaded = false;
    uint32_t sh_fin = 0;  // bit d: the coefficients of degrees 0..d are all finite
    bool sh_checked = false;

    for (int vi = 0; vi < nviews; ++vi) {
        const ViewParams& v = views[vi];
        const uint32_t rec = rec_base + (uint32_t)vi * n_pad + (uint32_t)g;
        // FP32 order key (also the near-plane test)
        const float z32 = __builtin_fmaf(v.V[6], mx, __builtin_fmaf(v.V[7], my, __builtin_fmaf(v.V[8], mz, v.tz_key)));
        bool vis = ok && z32 > NEAR_Z;
        uint32_t touched = 0, fb = 0;
        float4 r0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0}, r2 = {0, 0, 0, 0};
        uint2 bb = {0u, 0u}, tr = {0u, 0u};
        if (vis) {
            // camera-space centre, double-float: d = mu - t exactly, p = V d
            const df dX = two_sum(mx, -v.cam[0]), dY = two_sum(my, -v.cam[1]), dZ = two_sum(mz, -v.cam[2]);
            const df px = df_add(df_add(df_mulf(dX, v.V[0]), df_mulf(dY, v.V[1])), df_mulf(dZ, v.V[2]));
            const df py = df_add(df_add(df_mulf(dX, v.V[3]), df_mulf(dY, v.V[4])), df_mulf(dZ, v.V[5]));
            const df pz = df_add(df_add(df_mulf(dX, v.V[6]), df_mulf(dY, v.V[7])), df_mulf(dZ, v.V[8]));
            const float zc = pz.hi;
            // pixel centre of the Gaussian: u = fx x/z + cx, v = fy y/z + cy
            const df u = df_add(df_mulf(df_div(px, pz), v.fx), df{v.cx, 0.0f});
            const df w = df_add(df_mulf(df_div(py, pz), v.fy), df{v.cy, 0.0f});
            // start the SH loads now when the footprint can reach the image, so
            // they arrive during the EWA step: the footprint half-width is at
            // most 3.34 (f/z (1 + lim) max scale + 0.55) pixels
            {
                const float rb = 3.4f * (fmaxf(v.fx, v.fy) / zc * (1.0f + fmaxf(v.lim_x, v.lim_y)) * smax + 0.6f) + 1.0f;
                const bool maybe = u.hi > -rb && u.hi < (float)v.width + rb && w.hi > -rb && w.hi < (float)v.height + rb;
                if (maybe && !sh_loaded) {
                    load_sh<ST, DEG>(s, n, g, k);
                    sh_loaded = true;
                }
            }
            // EWA: T = J V with the Jacobian at the clamped direction; Sigma2D = (T M)(T M)^T + 0.3 I
            const float iz = 1.0f / zc;
            const float rx = fminf(fmaxf(px.hi * iz, -v.lim_x), v.lim_x);
            const float ry = fminf(fmaxf(py.hi * iz, -v.lim_y), v.lim_y);
            const float fxz = v.fx * iz, fyz = v.fy * iz;
            float T0[3], T1[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T0[j] = fxz * __builtin_fmaf(-rx, v.V[6 + j], v.V[j]);
                T1[j] = fyz * __builtin_fmaf(-ry, v.V[6 + j], v.V[3 + j]);
            }
            float m0[3], m1[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                m0[c] = __builtin_fmaf(T0[0], M[c], __builtin_fmaf(T0[1], M[3 + c], T0[2] * M[6 + c]));
                m1[c] = __builtin_fmaf(T1[0], M[c], __builtin_fmaf(T1[1], M[3 + c], T1[2] * M[6 + c]));
            }
            float a = __builtin_fmaf(m0[0], m0[0], __builtin_fmaf(m0[1], m0[1], m0[2] * m0[2])) + DILATION;
            float b = __builtin_fmaf(m0[0], m1[0], __builtin_fmaf(m0[1], m1[1], m0[2] * m1[2]));
            float c = __builtin_fmaf(m1[0], m1[0], __builtin_fmaf(m1[1], m1[1], m1[2] * m1[2])) + DILATION;
            const float ac = a * c;
            const float det = ac - b * b;
            float ca, cb, cc;
            if (!(det > ac * KAPPA_INV)) {
                // near-singular 2D covariance: its conic is recomputed in FP64
                // by conic_fp64 (listed below); a and c are sums of squares
                // and exact enough for the footprint
                ca = cb = cc = 0.0f;
                fb = 1;
            } else {
                const float id = 1.0f / det;
                ca = c * id;
                cb = -b * id;
                cc = a * id;
            }
            // conservative footprint: bounding box of the widened support ellipse
            const float ex = sqrtf(k2m * a), ey = sqrtf(k2m * c);
            vis = vis && __builtin_isfinite(u.hi) && __builtin_isfinite(w.hi) && __builtin_isfinite(ex) &&
                  __builtin_isfinite(ey) && __builtin_isfinite(ca) && __builtin_isfinite(cb) && __builtin_isfinite(cc);
            if (vis) {
                const float mg = 1.0f / 256.0f;
                // pixel i is inside when |i + 0.5 - u| <= ex
                const float fw = (float)v.width, fh = (float)v.height;
                const float xl = fminf(fmaxf(u.hi - ex - 0.5f - mg, -1.0f), fw);
                const float xr = fminf(fmaxf(u.hi + ex - 0.5f + mg, -1.0f), fw);
                const float yl = fminf(fmaxf(w.hi - ey - 0.5f - mg, -1.0f), fh);
                const float yr = fminf(fmaxf(w.hi + ey - 0.5f + mg, -1.0f), fh);
                const int x0 = max((int)ceilf(xl), 0), x1 = min((int)floorf(xr), v.width - 1);
                const int y0 = max((int)ceilf(yl), 0), y1 = min((int)floorf(yr), v.height - 1);
                if (x0 <= x1 && y0 <= y1) {
                    const int tx0 = x0 / v.tile_w, tx1 = x1 / v.tile_w;
                    const int ty0 = y0 / v.tile_h, ty1 = y1 / v.tile_h;
                    touched = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                    bb = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
                    tr = make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16),
                                    (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)(ty1 - ty0 + 1) << 16));
                }
            }
            if (touched) {
                if (!sh_loaded) {
                    load_sh<ST, DEG>(s, n, g, k);
                    sh_loaded = true;
                }
                // colour at the direction camera centre -> Gaussian
                const float dx = dX.hi, dy = dY.hi, dz = dZ.hi;
                const float dn = 1.0f / sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
                float rgb[3];
                sh_colour<DEG>(k, dx * dn, dy * dn, dz * dn, v.sh_degree, rgb);
                if (!sh_checked) {  // once per Gaussian, where the loads have landed
                    sh_fin = sh_finite<DEG>(k);
                    sh_checked = true;
                }
                // a non-finite SH coefficient of the degree in use drops the
                // Gaussian, as any other non-finite attribute does (and so
                // does a colour that overflows): every record's colour is finite
                const bool fin = ((sh_fin >> v.sh_degree) & 1u) && __builtin_isfinite(rgb[0]) &&
                                 __builtin_isfinite(rgb[1]) && __builtin_isfinite(rgb[2]);
                if (!fin) {
                    touched = 0;
                    fb = 0;
                    tr = make_uint2(0u, 0u);
                }
                r0 = make_float4(u.hi, w.hi, u.lo, w.lo);
                r1 = make_float4(-0.5f * LOG2E * ca, -LOG2E * cb, -0.5f * LOG2E * cc, L);
                r2 = make_float4(rgb[0], rgb[1], rgb[2], op);
            }
        }
        {
            // append near-singular visible Gaussians to the FP64 list (one atomic per wave)
            const bool lst = touched && fb;
            const uint64_t m = ballot(lst);
            if (m) {
                uint32_t base = 0;
                if ((threadIdx.x & 63) == (uint32_t)__builtin_ctzll(m))
                    base = atomicAdd(&o.cnt->fb_list, (uint32_t)__builtin_popcountll(m));
                base = readlane(base, __builtin_ctzll(m));
                const uint32_t pos = base + bits_below(m);
                if (lst && pos < o.fb_cap) o.fb_list[pos] = make_uint2(rec, (uint32_t)g);
            }
        }
        o.zkey[rec] = __float_as_uint(z32);
        if (touched) {
            Rec out;
            out.r0 = r0;
            out.r1 = r1;
            out.r2 = r2;
            out.bbox = bb;
            out.pad = make_uint2(0u, 0u);
            o.rec[rec] = out;
        }
        o.rect[rec] = tr;  // every record: whole-line, coalesced stores
        // per-block counts: wave sums, then one barrier (LDS slots alternate
        // between views so the next view cannot overwrite unread sums)
        const uint32_t s0 = wave_sum(touched), s1 = wave_sum(touched ? 1u : 0u), s2 = wave_sum(touched ? fb : 0u);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[vi & 1][wv][0] = s0;
            red[vi & 1][wv][1] = s1;
            red[vi & 1][wv][2] = s2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
            for (int j = 0; j < K1_THREADS / 64; ++j) {
                t0 += red[vi & 1][j][0];
                t1 += red[vi & 1][j][1];
                t2 += red[vi & 1][j][2];
            }
            const uint32_t blk = rec / K1_THREADS;
            o.blk_sum[blk] = t0;
            o.blk_vis[blk] = t1;
            o.blk_fb[blk] = t2;
            o.blk_view[blk] = view_base + (uint32_t)vi;
        }
    }
}

// Conic of a listed near-singular Gaussian, recomputed in FP64 from the
// FP32 inputs: Sigma2D, its determinant and its inverse; the exponent
// coefficients of the record are overwritten (log2 opacity kept).  Run by
// k_ranges: nothing between preprocess and the blend reads the coefficients.
__device__ void conic_fp64(const uint2 e, const ViewParams* __restrict__ views, const uint32_t* __restrict__ blk_view,
                           Rec* __restrict__ recs) {
    {
        const uint32_t rec = e.x;
        const int64_t g = e.y;
        const ViewParams& v = views[blk_view[rec / K1_THREADS]];
        const SceneView& s = v.scene;
        const int64_t N = s.n;
        const float mx = s.mean[g], my = s.mean[N + g], mz = s.mean[2 * N + g];
        float q[4], ls[3];
        if (s.storage == 0) {
            const float4* a = reinterpret_cast<const float4*>(s.attr);
            const float4 r = a[g], m = a[N + g];
            q[0] = r.x; q[1] = r.y; q[2] = r.z; q[3] = r.w;
            ls[0] = m.x; ls[1] = m.y; ls[2] = m.z;
        } else {
            float f[8];
            unpack8(reinterpret_cast<const uint4*>(s.attr)[g], f, s.storage);
            q[0] = f[0]; q[1] = f[1]; q[2] = f[2]; q[3] = f[3];
            ls[0] = f[4]; ls[1] = f[5]; ls[2] = f[6];
        }
        double abc[3];
        cov2d_fp64(q, ls, mx, my, mz, v, abc);
        const double d64 = abc[0] * abc[2] - abc[1] * abc[1];
        float4 r = recs[rec].r1;
        r.x = -0.5f * LOG2E * (float)(abc[2] / d64);
        r.y = -LOG2E * (float)(-abc[1] / d64);
        r.z = -0.5f * LOG2E * (float)(abc[0] / d64);
        recs[rec].r1 = r;
    }
}

// Counts are staged through LDS for the scans: coalesced loads, SCAN_ITEMS
// consecutive counts per thread summed from LDS (one pad word per 32 keeps
// those strided reads free of bank conflicts), offsets written back through
// LDS and stored coalesced.
constexpr int SCAN_STAGE = SCAN_CHUNK + SCAN_CHUNK / 32;
__device__ __forceinline__ int spad(int i) { return i + (i >> 5); }

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, unsigned long long* lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += lds[i];
    __syncthreads();
    return t;
}

// Multi-workgroup exclusive scans of per-block counts, chunk by chunk
// (SCAN_CHUNK counts per workgroup), in two kernels: chunk totals, then each
// chunk scanned from the sum of the totals before it.

// Totals of chunk blockIdx.x of `in` (and optionally of two more count arrays).
__global__ __launch_bounds__(SCAN_THREADS) void k_chunk_totals(const uint32_t* __restrict__ in, int n,
                                                               const uint32_t* __restrict__ in_a,
                                                               const uint32_t* __restrict__ in_b,
                                                               uint32_t* __restrict__ tot,
                                                               unsigned long long* __restrict__ tot_a,
                                                               uint32_t* __restrict__ tot_b) {
    __shared__ unsigned long long red64[SCAN_THREADS / 64];
    const int base = (int)blockIdx.x * SCAN_CHUNK;
    uint64_t s = 0, sa = 0, sb = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int i = base + r * SCAN_THREADS + (int)threadIdx.x;
        if (i < n) {
            s += in[i];
            if (in_a) sa += in_a[i];
            if (in_b) sb += in_b[i];
        }
    }
    s = block_sum_u64(s, red64);
    if (in_a) sa = block_sum_u64(sa, red64);
    if (in_b) sb = block_sum_u64(sb, red64);
    if (threadIdx.x == 0) {
        tot[blockIdx.x] = (uint32_t)s;
        if (tot_a) tot_a[blockIdx.x] = sa;
        if (tot_b) tot_b[blockIdx.x] = (uint32_t)sb;
    }
}

// Exclusive scan of chunk blockIdx.x of `in` into `out`, starting from the
// sum of the totals of the chunks before it.
__device__ void scan_chunk(const uint32_t* __restrict__ in, int n, const uint32_t* __restrict__ tot,
                           uint32_t* __restrict__ out, uint32_t* red, unsigned long long* red64, uint32_t* stage) {
    uint64_t p = 0;
    for (int c = (int)threadIdx.x; c < (int)blockIdx.x; c += SCAN_THREADS) p += tot[c];
    const uint32_t prefix = (uint32_t)block_sum_u64(p, red64);
    const int base = (int)blockIdx.x * SCAN_CHUNK;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int i = r * SCAN_THREADS + (int)threadIdx.x;
        stage[spad(i)] = base + i < n ? in[base + i] : 0u;
    }
    __syncthreads();
    uint32_t loc[SCAN_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        loc[j] = sum;
        sum += stage[spad((int)threadIdx.x * SCAN_ITEMS + j)];
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan<SCAN_THREADS>(sum, red, &total);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) stage[spad((int)threadIdx.x * SCAN_ITEMS + j)] = prefix + ex + loc[j];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int i = r * SCAN_THREADS + (int)threadIdx.x;
        if (base + i < n) out[base + i] = stage[spad(i)];
    }
}

// After preprocess (second kernel of the chunked scan): compaction offsets of
// the visible records; workgroup 0 also sets the totals V, D and FP64-fallback
// count and the overflow flag; every workgroup clears part of the per-frame
// accumulators of later kernels (digit totals, work queues, tile ranges).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_visible(const uint32_t* __restrict__ blk_vis, int nblk,
                                                               const uint32_t* __restrict__ tot_vis,
                                                               const unsigned long long* __restrict__ tot_dup,
                                                               const uint32_t* __restrict__ tot_fb, int nchunks,
                                                               uint32_t* __restrict__ blk_off, Counters* cnt,
                                                               uint32_t cap, ZeroList zl) {
    __shared__ uint32_t red[SCAN_THREADS / 64];
    __shared__ unsigned long long red64[SCAN_THREADS / 64];
    __shared__ uint32_t stage[SCAN_STAGE];
    scan_chunk(blk_vis, nblk, tot_vis, blk_off, red, red64, stage);
    if (blockIdx.x == 0) {
        uint64_t V = 0, D = 0, F = 0;
        for (int c = (int)threadIdx.x; c < nchunks; c += SCAN_THREADS) {
            V += tot_vis[c];
            D += tot_dup[c];
            F += tot_fb[c];
        }
        V = block_sum_u64(V, red64);
        D = block_sum_u64(D, red64);
        F = block_sum_u64(F, red64);
        if (threadIdx.x == 0) {
            cnt->D = D > 0xffffffffull ? 0xffffffffu : (uint32_t)D;
            cnt->visible = (uint32_t)V;
            cnt->fallbacks = (uint32_t)F;
            cnt->overflow = D > (uint64_t)cap ? 1u : 0u;
            cnt->fb_listed = cnt->fb_list;  // every preprocess launch has appended
            cnt->fb_list = 0u;                // the next frame appends from zero
        }
    }
#pragma unroll
    for (int k = 0; k < ZeroList::N; ++k)
        for (uint32_t i = blockIdx.x * SCAN_THREADS + threadIdx.x; i < zl.n[k]; i += gridDim.x * SCAN_THREADS)
            zl.p[k][i] = 0u;
}

// Emission offsets: exclusive scan of the duplicate counts of the
// depth-sorted visible Gaussians, per 256-element block (second kernel of the
// chunked scan).
// With `cnt`, workgroup 0 also stores the sum of the counts as the frame's
// duplicate count D (the count once tiles are culled), unless the frame
// overflowed: D then keeps the whole rectangles' count the buffers are grown to.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_dups(const uint32_t* __restrict__ blk_sum, int nblk,
                                                            const uint32_t* __restrict__ tot,
                                                            uint32_t* __restrict__ blk_off, int nchunks,
                                                            Counters* cnt) {
    __shared__ uint32_t red[SCAN_THREADS / 64];
    __shared__ unsigned long long red64[SCAN_THREADS / 64];
    __shared__ uint32_t stage[SCAN_STAGE];
    scan_chunk(blk_sum, nblk, tot, blk_off, red, red64, stage);
    if (cnt && blockIdx.x == 0) {
        uint64_t D = 0;
        for (int c = (int)threadIdx.x; c < nchunks; c += SCAN_THREADS) D += tot[c];
        D = block_sum_u64(D, red64);
        if (threadIdx.x == 0 && !cnt->overflow) cnt->D = (uint32_t)min(D, 0xffffffffull);
    }
}

// Tile rectangle (tx0 | ty0 << 16, nx | ny << 16) packed into one word as
// tx0 | ty0 << 8 | tx1 << 16 | ty1 << 24 (views of at most 256 x 256 tiles),
// and back.
__device__ __forceinline__ uint32_t pack_rect(uint2 r) {
    const uint32_t tx0 = r.x & 0xffffu, ty0 = r.x >> 16;
    return tx0 | (ty0 << 8) | ((tx0 + (r.y & 0xffffu) - 1u) << 16) | ((ty0 + (r.y >> 16) - 1u) << 24);
}
__device__ __forceinline__ uint2 unpack_rect(uint32_t p) {
    const uint32_t tx0 = p & 0xffu, ty0 = (p >> 8) & 0xffu, tx1 = (p >> 16) & 0xffu, ty1 = p >> 24;
    return make_uint2(tx0 | (ty0 << 16), (tx1 - tx0 + 1u) | ((ty1 - ty0 + 1u) << 16));
}

// Visible records, in record order, as (depth key, record) pairs, and with
// `ext` the packed tile rectangle as a third word that the depth passes carry
// along.  Four records per thread (16-byte loads): a workgroup covers four
// preprocess blocks, whose first compaction offset it starts from.
__global__ __launch_bounds__(K1_THREADS) void k_compact(const uint32_t* __restrict__ zkey,
                                                        const uint2* __restrict__ rect,
                                                        const uint32_t* __restrict__ blk_off, int nblk,
                                                        uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                        uint32_t* __restrict__ ext, const Counters* __restrict__ cnt,
                                                        const uint2* __restrict__ fb_list, uint32_t fb_cap,
                                                        const ViewParams* __restrict__ views,
                                                        const uint32_t* __restrict__ blk_view, Rec* __restrict__ recs) {
    __shared__ uint32_t red[K1_THREADS / 64];
    // the FP64 conics of the near-singular Gaussians (a few hundred per
    // frame), before anything reads the exponent coefficients
    const uint32_t nfb = min(cnt->fb_listed, fb_cap);
    for (uint32_t k = blockIdx.x * K1_THREADS + threadIdx.x; k < nfb; k += gridDim.x * K1_THREADS)
        conic_fp64(fb_list[k], views, blk_view, recs);
    const uint32_t nrec = (uint32_t)nblk * K1_THREADS;  // a multiple of 4
    const uint32_t r0 = (blockIdx.x * K1_THREADS + threadIdx.x) * 4u;
    uint4 z = make_uint4(0u, 0u, 0u, 0u), ra = z, rb = z;
    if (r0 < nrec) {  // a record is visible when its rectangle has tiles
        z = *reinterpret_cast<const uint4*>(zkey + r0);
        ra = *reinterpret_cast<const uint4*>(rect + r0);
        rb = *reinterpret_cast<const uint4*>(rect + r0 + 2);
    }
    // loaded with the inputs, not after the scan: one memory round trip less
    const uint32_t boff = (uint32_t)blockIdx.x * 4u < (uint32_t)nblk ? blk_off[blockIdx.x * 4] : 0u;
    const bool v0 = ra.y != 0u, v1 = ra.w != 0u, v2 = rb.y != 0u, v3 = rb.w != 0u;
    const uint32_t c = (uint32_t)v0 + (uint32_t)v1 + (uint32_t)v2 + (uint32_t)v3;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<K1_THREADS>(c, red, &tot);
    if (c) {
        uint32_t pos = boff + ex;
        if (ext) {
            if (v0) { key[pos] = z.x; val[pos] = r0; ext[pos] = pack_rect(make_uint2(ra.x, ra.y)); ++pos; }
            if (v1) { key[pos] = z.y; val[pos] = r0 + 1; ext[pos] = pack_rect(make_uint2(ra.z, ra.w)); ++pos; }
            if (v2) { key[pos] = z.z; val[pos] = r0 + 2; ext[pos] = pack_rect(make_uint2(rb.x, rb.y)); ++pos; }
            if (v3) { key[pos] = z.w; val[pos] = r0 + 3; ext[pos] = pack_rect(make_uint2(rb.z, rb.w)); }
        } else {
            if (v0) { key[pos] = z.x; val[pos] = r0; ++pos; }
            if (v1) { key[pos] = z.y; val[pos] = r0 + 1; ++pos; }
            if (v2) { key[pos] = z.z; val[pos] = r0 + 2; ++pos; }
            if (v3) { key[pos] = z.w; val[pos] = r0 + 3; }
        }
    }
}

// Tiles in a tile rectangle (tx0 | ty0 << 16, nx | ny << 16), and in a packed one.
__device__ __forceinline__ uint32_t rect_tiles(uint2 r) { return (r.y & 0xffffu) * (r.y >> 16); }
__device__ __forceinline__ uint32_t rect_count(uint32_t p) {
    return (((p >> 16) & 0xffu) - (p & 0xffu) + 1u) * ((p >> 24) - ((p >> 8) & 0xffu) + 1u);
}

// Per 256 depth-sorted visible Gaussians: the sum of their tile counts (zero
// past the visible count); workgroups stride over the nblk blocks.  The
// rectangles come packed (sorted_packed) or as two words (sorted_rect).
__global__ __launch_bounds__(K1_THREADS) void k_sorted_sums(const uint2* __restrict__ sorted_rect,
                                                            const uint32_t* __restrict__ sorted_packed,
                                                            const Counters* __restrict__ cnt, int nblk,
                                                            uint32_t* __restrict__ blk_sum) {
    __shared__ uint32_t red[K1_THREADS / 64];
    const uint32_t V = cnt->visible;
    for (uint32_t b = blockIdx.x; b < (uint32_t)nblk; b += gridDim.x) {
        if (b * K1_THREADS >= V) {  // uniform: empty block
            if (threadIdx.x == 0) blk_sum[b] = 0u;
            continue;
        }
        const uint32_t i = b * K1_THREADS + threadIdx.x;
        uint32_t t = 0;
        if (i < V) t = rect_tiles(sorted_packed ? unpack_rect(sorted_packed[i]) : sorted_rect[i]);
        const uint32_t s = block_sum<K1_THREADS>(t, red);
        if (threadIdx.x == 0) blk_sum[b] = s;
    }
}

// ---------------------------------------------------------------- duplicate
// One entry per (Gaussian, overlapped tile), Gaussians taken in depth order,
// tiles row-major over the Gaussian's tile rectangle: tile word = global tile
// id, value = record, and (when asked) the depth word, so that the entry's
// 64-bit key is (tile id << 32) | depth bits.  Load-balanced: the threads of a
// workgroup write consecutive entries of their 256 Gaussians' output range,
// each finding its Gaussian by binary search over the LDS prefix sums.
template <bool DEPTH>
__global__ __launch_bounds__(K1_THREADS) void k_duplicate(const uint32_t* __restrict__ sorted_rec,
                                                          const uint2* __restrict__ sorted_rect,
                                                          const uint32_t* __restrict__ sorted_packed,
                                                          const uint32_t* __restrict__ zkey,
                                                          const uint32_t* __restrict__ blk_off,
                                                          const uint32_t* __restrict__ blk_view,
                                                          const Counters* __restrict__ cnt, uint32_t cap,
                                                          const ViewParams* __restrict__ views,
                                                          uint32_t* __restrict__ tile_out,
                                                          uint32_t* __restrict__ val_out,
                                                          uint32_t* __restrict__ depth_out) {
    __shared__ uint32_t red[K1_THREADS / 64];
    __shared__ uint32_t pre[K1_THREADS + 1];  // inclusive prefix of tile counts, pre[0] = 0
    __shared__ uint32_t srec[K1_THREADS];
    __shared__ uint32_t sx0[K1_THREADS], stx[K1_THREADS], snx[K1_THREADS], stb[K1_THREADS];
    __shared__ float sinx[K1_THREADS];
    __shared__ uint32_t own[K1_THREADS];           // round-tagged owner marks of the output slots
    __shared__ uint32_t wmax[K1_THREADS / 64];
    static_assert(K1_THREADS == 256, "owner marks keep the Gaussian index in 8 bits");
    const uint32_t i = blockIdx.x * K1_THREADS + threadIdx.x;
    const uint32_t V = cnt->visible;
    uint32_t rec = 0, t = 0;
    uint2 tr = make_uint2(0u, 0u);
    if (i < V) {
        rec = sorted_rec[i];
        // tile rectangle in depth order: carried packed through the depth
        // passes, or gathered by the last one
        tr = sorted_packed ? unpack_rect(sorted_packed[i]) : sorted_rect[i];
        t = rect_tiles(tr);
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<K1_THREADS>(t, red, &tot);
    if (cnt->overflow || tot == 0) return;  // uniform across the workgroup
    pre[threadIdx.x + 1] = ex + t;
    if (threadIdx.x == 0) pre[0] = 0;
    own[threadIdx.x] = 0u;
    srec[threadIdx.x] = rec;
    if (t) {
        const ViewParams& v = views[blk_view[rec / K1_THREADS]];
        const uint32_t nx = tr.y & 0xffffu;
        sx0[threadIdx.x] = tr.x & 0xffffu;
        snx[threadIdx.x] = nx;
        sinx[threadIdx.x] = 1.0f / (float)nx;
        stb[threadIdx.x] = v.tile_base;
        // tiles_x of the view, packed with the first row
        stx[threadIdx.x] = (tr.x >> 16) | ((uint32_t)v.tiles_x << 16);
    }
    __syncthreads();
    const uint32_t base = blk_off[blockIdx.x];
    // Output slots in rounds of 256.  The owner of slot j is the last
    // Gaussian e whose first slot is at or before j: every Gaussian marks its
    // first slot in the round it falls in with (round << 8) | e, and a
    // prefix maximum over the round's slots, started from the previous
    // round's last owner, gives each slot's owner.  Marks of earlier rounds
    // are smaller than any tag of the current one, so `own` is never cleared.
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;  // owner of the slot before the round
    for (uint32_t j0 = 0, m = 0; j0 < tot; j0 += K1_THREADS, ++m) {
        if (t && (ex >> 8) == m) own[ex & (K1_THREADS - 1)] = (m << 8) | threadIdx.x;
        __syncthreads();
        const uint32_t incl = wave_incl_max(own[threadIdx.x]);
        if (lane == 63) wmax[w] = incl;
        __syncthreads();
        uint32_t o = max(incl, (m << 8) | carry), all = (m << 8) | carry;
#pragma unroll
        for (uint32_t v = 0; v < K1_THREADS / 64; ++v) {
            const uint32_t x = wmax[v];
            if (v < w) o = max(o, x);
            all = max(all, x);
        }
        carry = all & 0xffu;
        const uint32_t j = j0 + threadIdx.x;
        if (j >= tot) continue;
        const uint32_t e = o & 0xffu;
        const uint32_t k = j - pre[e];
        const uint32_t nx = snx[e];
        // k / nx through the FP32 reciprocal, corrected to the exact quotient
        uint32_t q = (uint32_t)((float)k * sinx[e]);
        if (q * nx > k) --q;
        if ((q + 1) * nx <= k) ++q;
        const uint32_t ty = (stx[e] & 0xffffu) + q, tx = sx0[e] + (k - q * nx);
        const uint32_t tiles_x = stx[e] >> 16;
        const uint32_t r = srec[e];
        tile_out[base + j] = stb[e] + ty * tiles_x + tx;
        val_out[base + j] = r;
        if (DEPTH) depth_out[base + j] = zkey[r];
    }
}


// ------------------------------------------------- tighter tile culling
// Whether a Gaussian can reach the skip threshold (alpha >= 1/255) at some
// pixel centre of a tile: the exact maximum of its exponent
// e(d) = A dx^2 + B dx dy + C dy^2 + L over the rectangle of the tile's pixel
// centres inside the frame (as in the blend's block test: the centre when it
// lies inside, else the better of the two faces facing it, each maximised at a
// clamped stationary point), compared with the threshold less the blend's
// margin, so a dropped tile is one every pixel of it would skip.  Plain FP32
// operations only (IEEE division, no fused or approximate ones), in this
// order, so a CPU reference reproduces every decision bit for bit.
// (ox, oy): the tile's pixel origin; (cw, ch): its pixels inside the frame.
__device__ __forceinline__ bool tile_reaches(float uhi, float vhi, float ulo, float vlo, float A, float B, float C,
                                             float L, float ox, float oy, float cw, float ch) {
    const float u = (uhi - ox) + ulo, v = (vhi - oy) + vlo;
    const float dx0 = 0.5f - u, dx1 = (cw - 0.5f) - u;
    const float dy0 = 0.5f - v, dy1 = (ch - 0.5f) - v;
    if (!(A < 0.0f && C < 0.0f && B * B < (4.0f * A) * C)) return true;  // not concave: keep it
    float q = 0.0f;
    if (!(dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f)) {
        const float cx = dx1 < 0.0f ? dx1 : dx0;
        const float sy = fminf(fmaxf((-B * cx) / (2.0f * C), dy0), dy1);
        const float ex = (A * cx + B * sy) * cx + (C * sy) * sy;
        const float cy = dy1 < 0.0f ? dy1 : dy0;
        const float sx = fminf(fmaxf((-B * cy) / (2.0f * A), dx0), dx1);
        const float ey = (C * cy + B * sx) * cy + (A * sx) * sx;
        q = fmaxf(ex, ey);
    }
    const float r2 = fmaxf(dx0 * dx0, dx1 * dx1) + fmaxf(dy0 * dy0, dy1 * dy1);
    const float margin = 0.02f + (1e-5f * ((fabsf(A) + fabsf(B)) + fabsf(C))) * r2;
    return !(q + L < LOG2_ALPHA_MIN - margin);  // keeps NaN
}

// The tile-culled duplicates: the same enumeration of (Gaussian, tile in its
// rectangle) slots as k_duplicate, each kept only when tile_reaches says so.
// COUNT: per block of 256 depth-ordered Gaussians, the number of kept entries
// (block_cnt).  Otherwise the kept entries are written in slot order,
// compacted, from the block's offset (blk_off, the exclusive scan of the
// counts).  The records already hold the FP64 conics of the near-singular
// Gaussians (patched by k_compact), so both launches test the final
// coefficients.
template <bool COUNT, bool DEPTH>
__global__ __launch_bounds__(K1_THREADS) void k_duplicate_culled(
    const uint32_t* __restrict__ sorted_rec, const uint32_t* __restrict__ sorted_packed,
    const uint32_t* __restrict__ zkey, const uint32_t* __restrict__ blk_off, uint32_t* __restrict__ block_cnt,
    const uint32_t* __restrict__ blk_view, const Counters* __restrict__ cnt, const ViewParams* __restrict__ views,
    const Rec* __restrict__ recs, int tile_w, int tile_h, uint32_t* __restrict__ tile_out,
    uint32_t* __restrict__ val_out, uint32_t* __restrict__ depth_out) {
    __shared__ uint32_t red[K1_THREADS / 64];
    __shared__ uint32_t pre[K1_THREADS + 1];
    __shared__ uint32_t srec[K1_THREADS], spk[K1_THREADS], stb[K1_THREADS], swh[K1_THREADS];
    __shared__ float4 sr0[K1_THREADS], sr1[K1_THREADS];
    __shared__ uint32_t own[K1_THREADS];
    __shared__ uint32_t wmax[K1_THREADS / 64];
    const uint32_t i = blockIdx.x * K1_THREADS + threadIdx.x;
    const uint32_t V = cnt->visible;
    uint32_t rec = 0, p = 0, t = 0;
    if (i < V) {
        rec = sorted_rec[i];
        p = sorted_packed[i];
        t = rect_count(p);
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<K1_THREADS>(t, red, &tot);
    if (!COUNT && (cnt->overflow || tot == 0)) return;  // uniform across the workgroup
    pre[threadIdx.x + 1] = ex + t;
    if (threadIdx.x == 0) pre[0] = 0;
    own[threadIdx.x] = 0u;
    srec[threadIdx.x] = rec;
    spk[threadIdx.x] = p;
    if (t) {
        const ViewParams& v = views[blk_view[rec / K1_THREADS]];
        stb[threadIdx.x] = v.tile_base;
        swh[threadIdx.x] = (uint32_t)v.width | ((uint32_t)v.height << 16);
        sr0[threadIdx.x] = recs[rec].r0;
        sr1[threadIdx.x] = recs[rec].r1;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t base = COUNT ? 0u : blk_off[blockIdx.x];
    uint32_t kept_before = 0;  // kept entries of this block in earlier rounds
    uint32_t carry = 0;
    for (uint32_t j0 = 0, m = 0; j0 < tot; j0 += K1_THREADS, ++m) {
        if (t && (ex >> 8) == m) own[ex & (K1_THREADS - 1)] = (m << 8) | threadIdx.x;
        __syncthreads();
        const uint32_t incl = wave_incl_max(own[threadIdx.x]);
        if (lane == 63) wmax[w] = incl;
        __syncthreads();
        uint32_t o = max(incl, (m << 8) | carry), all = (m << 8) | carry;
#pragma unroll
        for (uint32_t vv = 0; vv < K1_THREADS / 64; ++vv) {
            const uint32_t x = wmax[vv];
            if (vv < w) o = max(o, x);
            all = max(all, x);
        }
        carry = all & 0xffu;
        const uint32_t j = j0 + threadIdx.x;
        bool keep = false;
        uint32_t tile = 0, r = 0;
        if (j < tot) {
            const uint32_t e = o & 0xffu;
            const uint32_t k = j - pre[e];
            const uint32_t pk = spk[e];
            const uint32_t x0 = pk & 0xffu, y0 = (pk >> 8) & 0xffu;
            const uint32_t nx = ((pk >> 16) & 0xffu) - x0 + 1u;
            const uint32_t q = k / nx;
            const uint32_t ty = y0 + q, tx = x0 + (k - q * nx);
            const uint32_t wh = swh[e];
            const int W = (int)(wh & 0xffffu), H = (int)(wh >> 16);
            const int px = (int)tx * tile_w, py = (int)ty * tile_h;
            const float4 a = sr0[e], c = sr1[e];
            keep = tile_reaches(a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w, (float)px, (float)py,
                                (float)min(tile_w, W - px), (float)min(tile_h, H - py));
            const int tiles_x = (W + tile_w - 1) / tile_w;
            tile = stb[e] + ty * (uint32_t)tiles_x + tx;
            r = srec[e];
        }
        uint32_t kept_round;
        const uint32_t kex = block_excl_scan<K1_THREADS>(keep ? 1u : 0u, red, &kept_round);
        if (!COUNT && keep) {
            const uint32_t pos = base + kept_before + kex;
            tile_out[pos] = tile;
            val_out[pos] = r;
            if (DEPTH) depth_out[pos] = zkey[r];
        }
        kept_before += kept_round;
    }
    if (COUNT && threadIdx.x == 0) block_cnt[blockIdx.x] = kept_before;
}

// ------------------------------------------------------------- radix sort
// One pass sorts (key, value[, extra]) triples stably by an 8-bit (or
// narrower) digit of the key.  The count comes from the device counters
// (which = 0: duplicates D, 1: visible Gaussians V) and is split into nb
// contiguous segments, one per workgroup, of a whole number of 2048-key
// chunks.  upsweep: digit histogram per segment; scan: exclusive offsets over
// (digit, segment); downsweep: rank (wave ballots + per-wave LDS counters)
// and scatter.

// Three-pass depth sort: 9-bit digits of (key - base), base = the smallest
// visible key with its low 9 bits cleared (so the first pass, run before the
// smallest key is known, takes the key's own low 9 bits), when the keys span
// less than 2^27; wider frames are flagged and redone with the four 8-bit
// passes of the whole key.
constexpr int DEPTH3_BITS = 27;
__device__ __forceinline__ bool depth_wide(uint32_t lo, uint32_t hi) {
    return lo <= hi && ((hi - (lo & ~511u)) >> DEPTH3_BITS) != 0u;
}
// Digit base of a pass: fixed passes (adapt < 0) and the first adaptive pass
// take the key as it is; later adaptive passes subtract the base from the
// smallest and largest keys in zr, and are skipped (false) in a wide frame.
__device__ __forceinline__ bool pass_digit(int adapt, const uint32_t* zr, uint32_t* kbase) {
    *kbase = 0u;
    if (adapt <= 0) return true;
    const uint32_t lo = zr[0], hi = zr[1];
    if (depth_wide(lo, hi)) return false;
    if (lo <= hi) *kbase = lo & ~511u;
    return true;
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ uint32_t sort_count(const Counters* cnt, int which, uint32_t cap) {
    if (which == 1) return min(cnt->visible, cap);
    return cnt->overflow ? 0u : min(cnt->D, cap);
}
// Segment of workgroup `wg` of a pass: consecutive workgroup ids go
// round-robin to the 8 XCDs, so XCD x is given a contiguous run of segments
// (the runs of one digit written by neighbouring segments then meet in one
// L2 and leave it as whole cache lines).
__device__ __forceinline__ int xcd_segment(int wg, int nb) {
    const int per = nb >> 3, rem = nb & 7, x = wg & 7;
    return x * per + min(x, rem) + (wg >> 3);
}
__device__ __forceinline__ uint64_t segment_len(uint32_t D, int nb) {
    const uint64_t per = ((uint64_t)D + nb - 1) / nb;
    return (per + SORT_CHUNK - 1) / SORT_CHUNK * SORT_CHUNK;
}
// The segment of workgroup wg: the segments that hold keys are spread over
// the XCDs in contiguous runs, the empty ones keep their own index.
__device__ __forceinline__ int pass_segment(uint32_t D, int nb, int wg) {
    const uint64_t per = segment_len(D, nb);
    const int nact = per ? (int)min((uint64_t)nb, ((uint64_t)D + per - 1) / per) : 0;
    return wg < nact ? xcd_segment(wg, nact) : wg;
}
__device__ __forceinline__ void segment(uint32_t D, int nb, int b, uint32_t* beg, uint32_t* end) {
    const uint64_t per = segment_len(D, nb);
    const uint64_t s = min((uint64_t)D, per * (uint64_t)b);
    *beg = (uint32_t)s;
    *end = (uint32_t)min((uint64_t)D, s + per);
}

// Digit counts of one segment: hist[d * nb + b] = keys of digit d in segment
// b, pre[d * nb + b] = keys of digits below d in segment b (the segment's
// exclusive digit prefix).  Summed over segments, pre gives each digit's global
// start, so no kernel needs device-wide atomics on the 256 digit totals.
template <int NDIG, bool MINMAX>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_upsweep(const uint32_t* __restrict__ keys,
                                                               const Counters* __restrict__ cnt, int which,
                                                               uint32_t cap, int shift, int bits, int adapt,
                                                               const uint32_t* __restrict__ zr,
                                                               uint32_t* __restrict__ hist, int nb,
                                                               uint32_t* __restrict__ segmm) {
    static_assert(NDIG % SORT_THREADS == 0, "whole digits per thread");
    constexpr int DPT = NDIG / SORT_THREADS;  // digits per thread
    // NH sub-histograms, rows of NDIG+1 words so that the copies of one digit
    // sit in different LDS banks.  8-bit digits: one per wave and lane
    // residue mod 4, so that keys of one digit in one row of 64 (the leading
    // digit of the whole depth key is nearly constant) meet at most 16 to an
    // address; 9-bit digits (of the key less the smallest key, spread over
    // many values in every pass): one per wave
    constexpr int NW = SORT_THREADS / 64, LPW = NDIG > 256 ? 1 : 4, NH = NW * LPW, ROW = NDIG + 1;
    __shared__ uint32_t h[NH * ROW];
    __shared__ uint32_t wlo[NW], whi[NW];
    uint32_t kbase;
    if (!pass_digit(adapt, zr, &kbase)) return;  // uniform: a wide frame, redone with four passes
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < NH * ROW; i += SORT_THREADS) h[i] = 0u;
    __syncthreads();
    uint32_t beg, end;
    const uint32_t D = sort_count(cnt, which, cap);
    const int seg = pass_segment(D, nb, (int)blockIdx.x);
    segment(D, nb, seg, &beg, &end);
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t* hrow = h + (w * LPW + (lane & (LPW - 1))) * ROW;
    uint32_t lo = 0xffffffffu, hi = 0u;  // MINMAX: the segment's smallest and largest key
    // each wave walks blocks of 8 rows of 64 keys (8 loads in flight per lane)
    constexpr int U = 8;
    for (uint32_t blk = beg + (uint32_t)w * 64 * U; blk < end; blk += SORT_THREADS * U) {
        uint32_t kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = blk + u * 64 + lane;
            kk[u] = keys[i < end ? i : beg];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (blk + u * 64 + lane < end) {
                atomicAdd(&hrow[((kk[u] - kbase) >> shift) & mask], 1u);
                if (MINMAX) {
                    lo = min(lo, kk[u]);
                    hi = max(hi, kk[u]);
                }
            }
    }
    if (MINMAX) {
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane == 0) {
            wlo[w] = lo;
            whi[w] = hi;
        }
    }
    __syncthreads();
    if (MINMAX && threadIdx.x == 0) {
#pragma unroll
        for (int v = 1; v < NW; ++v) {
            lo = min(lo, wlo[v]);
            hi = max(hi, whi[v]);
        }
        segmm[2 * seg] = lo;
        segmm[2 * seg + 1] = hi;
    }
    // thread t: digits t DPT .. t DPT + DPT - 1
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int d = t * DPT + j;
        uint32_t x = 0;
#pragma unroll
        for (int k = 0; k < NH; ++k) x += h[k * ROW + d];
        if (d <= (int)mask) hist[(size_t)d * nb + seg] = x;
    }
}

// One workgroup per digit: the digit's exclusive offsets over the segments
// (within the digit) and its total.  The four waves take consecutive quarters of the digit's row
// (NJ * 64 segments each) and learn the totals of the quarters before theirs
// through LDS.
template <int NJ>
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ dtot,
                                                   int nb, int ndig, int adapt, uint32_t* __restrict__ zr,
                                                   const uint32_t* __restrict__ segmm, Counters* cnt) {
    __shared__ uint32_t qsum[4], qpre[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int d = blockIdx.x;
    if (adapt == 0 && d == ndig) {
        // the extra workgroup of the first pass of the three-pass depth sort:
        // the smallest and largest key over the segments; a frame whose keys
        // span 2^27 or more is flagged for the four-pass sort
        uint32_t lo = 0xffffffffu, hi = 0u;
        for (int i = threadIdx.x; i < nb; i += 256) {
            lo = min(lo, segmm[2 * i]);
            hi = max(hi, segmm[2 * i + 1]);
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane == 0) {
            qsum[w] = lo;
            qpre[w] = hi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int v = 1; v < 4; ++v) {
                lo = min(lo, qsum[v]);
                hi = max(hi, qpre[v]);
            }
            zr[0] = lo;
            zr[1] = hi;
            if (depth_wide(lo, hi)) atomicOr(&cnt->overflow, 2u);
        }
        return;
    }
    if (d >= ndig) return;  // whole workgroup exits together
    uint32_t kbase;
    if (!pass_digit(adapt, zr, &kbase)) return;  // uniform
    uint32_t* row = hist + (size_t)d * nb;
    const int j0 = w * NJ * 64;
    uint32_t x[NJ];  // 4 * NJ * 64 >= nb
    uint32_t mine = 0;
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        const int j = j0 + q * 64 + lane;
        x[q] = j < nb ? row[j] : 0u;
        mine += x[q];
    }
    const uint32_t ws = wave_sum(mine);
    if (lane == 0) qsum[w] = ws;
    __syncthreads();
    if (threadIdx.x == 0) dtot[d] = qsum[0] + qsum[1] + qsum[2] + qsum[3];
    uint32_t running = 0;
    for (int v = 0; v < w; ++v) running += qsum[v];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        if (j0 + q * 64 >= nb) break;
        const int j = j0 + q * 64 + lane;
        const uint32_t inc = wave_incl_scan(x[q]);
        if (j < nb) row[j] = running + inc - x[q];
        running += readlane(inc, 63);
    }
}

// Chunks of 2048 keys are ranked (per-wave ballot match + per-wave digit
// counters), staged in LDS in chunk-local digit order, and written out so that
// consecutive threads store consecutive positions of each digit run.  NT
// threads: 512 for the 9-bit depth digits (a digit per thread, four rounds
// of ranking per wave instead of eight: one chunk per workgroup, so the
// launch lasts about one workgroup's chain of rounds), else 256.
// SUMS (last depth pass): each Gaussian's tile rectangle is gathered once
// here and written in depth order, so that k_sorted_sums and k_duplicate read
// it contiguously instead of gathering by record.
template <bool EXTRA, bool SUMS, int NDIG, int NT>
__global__ __launch_bounds__(NT) void k_sort_downsweep(
    const uint32_t* __restrict__ skey, const uint32_t* __restrict__ sval, const uint32_t* __restrict__ sext,
    uint32_t* __restrict__ dkey, uint32_t* __restrict__ dval, uint32_t* __restrict__ dext,
    const Counters* __restrict__ cnt, int which, uint32_t cap, int shift, int bits, int adapt,
    const uint32_t* __restrict__ zr, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot, int nb,
    const uint2* __restrict__ rsrc, uint2* __restrict__ rdst) {
    static_assert(NDIG % NT == 0, "whole digits per thread");
    constexpr int DPT = NDIG / NT;  // digits per thread
    constexpr int NW = NT / 64;
    constexpr int ROUNDS = SORT_CHUNK / NT;
    __shared__ uint32_t base[NDIG];    // global position of the next key of each digit
    __shared__ uint32_t lstart[NDIG];  // chunk-local start of each digit
    __shared__ uint32_t wcnt[NW][NDIG];
    __shared__ uint32_t red[NW];
    __shared__ uint32_t lkey[SORT_CHUNK];
    __shared__ uint32_t lval[SORT_CHUNK];
    __shared__ uint32_t lext[EXTRA ? SORT_CHUNK : 1];
    __shared__ uint2 lrect[SUMS ? SORT_CHUNK : 1];
    uint32_t kbase;
    if (!pass_digit(adapt, zr, &kbase)) return;  // uniform: a wide frame, redone with four passes
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t beg, end;
    const uint32_t D = sort_count(cnt, which, cap);
    const int seg = pass_segment(D, nb, (int)blockIdx.x);
    segment(D, nb, seg, &beg, &end);
    // the keys of the next chunk are loaded while the current one is ranked
    // (the first chunk's while the digit starts are formed)
    uint32_t nk[ROUNDS], nv[ROUNDS], ne[ROUNDS];
    auto load_chunk = [&](uint32_t c) {
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const uint32_t idx = c + (uint32_t)(w * (SORT_CHUNK / NW) + r * 64 + lane);
            const uint32_t ic = idx < end ? idx : c;  // clamped: loads never depend on a branch
            nk[r] = skey[ic];
            nv[r] = sval[ic];
            ne[r] = EXTRA ? sext[ic] : 0u;
        }
    };
    if (beg < end) load_chunk(beg);
    // a digit's first position: the totals of the digits below it (scanned
    // here from the per-digit totals) plus its offset in this segment
    {
        uint32_t tt[DPT], ts = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = t * DPT + j;
            tt[j] = d <= (int)mask ? dtot[d] : 0u;
            ts += tt[j];
        }
        uint32_t all;
        uint32_t st = block_excl_scan<NT>(ts, red, &all);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = t * DPT + j;
            base[d] = d <= (int)mask ? st + hist[(size_t)d * nb + seg] : 0u;
            st += tt[j];
        }
    }
    for (uint32_t chunk = beg; chunk < end; chunk += SORT_CHUNK) {
#pragma unroll
        for (int j = 0; j < NW; ++j)
#pragma unroll
            for (int q = 0; q < DPT; ++q) wcnt[j][t * DPT + q] = 0u;
        __syncthreads();
        uint32_t dig[ROUNDS], rank[ROUNDS], ek[ROUNDS], ev[ROUNDS], ee[ROUNDS];
        uint2 er[ROUNDS];
        bool ok[ROUNDS];
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            ek[r] = nk[r];
            ev[r] = nv[r];
            ee[r] = ne[r];
        }
        if (chunk + SORT_CHUNK < end) load_chunk(chunk + SORT_CHUNK);
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const uint32_t idx = chunk + (uint32_t)(w * (SORT_CHUNK / NW) + r * 64 + lane);
            ok[r] = idx < end;
            const uint32_t key = ek[r];
            if constexpr (SUMS) er[r] = rsrc[ev[r]];
            const uint32_t d = ((key - kbase) >> shift) & mask;
            dig[r] = d;
            uint64_t m = ballot(ok[r]);
            for (int b = 0; b < bits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bl = ballot(bit);
                m &= bit ? bl : ~bl;
            }
            const uint32_t prior = (uint32_t)__builtin_popcountll(m & lt);
            uint32_t cur = 0;
            if (ok[r]) cur = wcnt[w][d];
            rank[r] = cur + prior;
            if (ok[r] && prior == 0) wcnt[w][d] = cur + (uint32_t)__builtin_popcountll(m);
        }
        __syncthreads();
        // digits t DPT ..: chunk-local start, then per-wave local offsets
        uint32_t c[DPT], csum = 0;
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            c[q] = 0;
#pragma unroll
            for (int j = 0; j < NW; ++j) c[q] += wcnt[j][t * DPT + q];
            csum += c[q];
        }
        uint32_t tot;
        uint32_t ls = block_excl_scan<NT>(csum, red, &tot);
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int d = t * DPT + q;
            lstart[d] = ls;
            uint32_t acc = ls;
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const uint32_t x = wcnt[j][d];
                wcnt[j][d] = acc;
                acc += x;
            }
            ls += c[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            if (ok[r]) {
                const uint32_t l = wcnt[w][dig[r]] + rank[r];
                lkey[l] = ek[r];
                lval[l] = ev[r];
                if (EXTRA) lext[l] = ee[r];
                if constexpr (SUMS) lrect[l] = er[r];
            }
        }
        __syncthreads();
        for (uint32_t l = (uint32_t)t; l < tot; l += NT) {
            const uint32_t k = lkey[l];
            const uint32_t d = ((k - kbase) >> shift) & mask;
            const uint32_t pos = base[d] + (l - lstart[d]);
            if (pos < D) {
                const uint32_t vv = lval[l];
                dkey[pos] = k;
                dval[pos] = vv;
                if (EXTRA) dext[pos] = lext[l];
                if constexpr (SUMS) rdst[pos] = lrect[l];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DPT; ++q) base[t * DPT + q] += c[q];
    }
}

// ------------------------------------------------------------------ ranges

// Tile boundaries in the sorted tile words; the ranges array was cleared by
// k_scan_visible, so tiles without entries stay [0, 0).  The frame's counters
// are final here: one thread also stores them to the host-visible block the
// host reads after the frame (no separate copy).
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tile, const Counters* __restrict__ cnt,
                                                uint32_t cap, uint2* __restrict__ ranges, Counters* host_cnt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *host_cnt = *cnt;
    const uint32_t D = sort_count(cnt, 0, cap);
    // each wave takes 256 consecutive words per step, four per lane (one
    // 16-byte load); neighbours come from the adjacent lanes, and across the
    // step's edges from one extra load
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * 4u;
    for (uint32_t c = ((blockIdx.x * 256u + threadIdx.x) >> 6) * 256u; c < D; c += nwaves * 256u) {
        const uint32_t i0 = c + (uint32_t)lane * 4u;
        uint32_t e[4];
        if (i0 + 3u < D) {
            const uint4 q = *reinterpret_cast<const uint4*>(tile + i0);
            e[0] = q.x; e[1] = q.y; e[2] = q.z; e[3] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) e[k] = i0 + k < D ? tile[i0 + k] : 0xffffffffu;
        }
        uint32_t prev = __shfl_up(e[3], 1, 64), next = __shfl_down(e[0], 1, 64);
        if (lane == 0) prev = c > 0u ? tile[c - 1u] : 0xffffffffu;
        if (lane == 63) next = c + 256u < D ? tile[c + 256u] : 0xffffffffu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = i0 + (uint32_t)k;
            if (i < D) {
                const uint32_t t = e[k];
                const uint32_t p = k > 0 ? e[k - 1] : prev, n = k < 3 ? e[k + 1] : next;
                if (i == 0u || p != t) ranges[t].x = i;
                if (i + 1u == D || n != t) ranges[t].y = i + 1u;
            }
        }
    }
}

// ---------------------------------------------------- binned tile digit
// The most significant digit of the (tile | depth) key, the tile id, placed
// by counting instead of by radix passes over the duplicates: the Gaussians
// arrive in depth order, and entry (g, t) belongs at
//   start(t) + #{Gaussians before g, in depth order, whose rectangle holds t}.
// The count over whole blocks of BIN_BLOCK Gaussians comes from per-block
// tile histograms (a 2D difference array over the tile grid: +1/-1 at the
// four corners of each rectangle, then 2D prefix sums) and their prefixes
// over blocks.  Entries are emitted in their depth-first order, BIN_PAIRS per
// workgroup (so a few large near Gaussians do not load one workgroup): a
// workgroup recounts the Gaussians of its block before its first round,
// and inside a round of 256 Gaussians the waves' column and row ballots give,
// per tile, the lanes whose rectangles hold it.  Each entry is written
// straight to its sorted position; the tile ranges fall out of the tile
// starts.  Single view, tile grid of at most BIN_GRID_MAX cells.

// Inclusive 2D prefix sums of an h1 x w1 grid (row-major, w1 <= 256) held in
// LDS, by a workgroup of 256 threads: rows (one wave per row, DPP scans), then
// columns (one thread per column, eight rows in flight).
__device__ void grid_prefix2d(uint32_t* g, int w1, int h1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int y = w; y < h1; y += 4) {
        uint32_t carry = 0;
        for (int c0 = 0; c0 < w1; c0 += 64) {
            const int x = c0 + lane;
            const uint32_t v = x < w1 ? g[y * w1 + x] : 0u;
            const uint32_t sc = wave_incl_scan(v) + carry;
            if (x < w1) g[y * w1 + x] = sc;
            carry = readlane(sc, 63);
        }
    }
    __syncthreads();
    const int x = threadIdx.x;
    if (x < w1) {
        uint32_t run = 0;
        int y = 0;
        for (; y + 8 <= h1; y += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = g[(y + k) * w1 + x];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                run += v[k];
                g[(y + k) * w1 + x] = run;
            }
        }
        for (; y < h1; ++y) {
            run += g[y * w1 + x];
            g[y * w1 + x] = run;
        }
    }
    __syncthreads();
}

// Adds one packed tile rectangle to the 2D difference grid g (stride w1).
// Corners in the extra column x = tiles_x or row y = tiles_y are left out:
// they only affect cells outside the tile grid, which nothing reads (and
// rectangles clamped to the frame's right or bottom edge would all meet
// there).
__device__ __forceinline__ void grid_add_rect(uint32_t* g, int w1, int tiles_x, int tiles_y, uint32_t p) {
    const int x0 = (int)(p & 0xffu), y0 = (int)((p >> 8) & 0xffu), x1 = (int)((p >> 16) & 0xffu) + 1,
              y1 = (int)(p >> 24) + 1;
    atomicAdd(&g[y0 * w1 + x0], 1u);
    if (x1 < tiles_x) atomicAdd(&g[y0 * w1 + x1], 0xffffffffu);
    if (y1 < tiles_y) {
        atomicAdd(&g[y1 * w1 + x0], 0xffffffffu);
        if (x1 < tiles_x) atomicAdd(&g[y1 * w1 + x1], 1u);
    }
}

// The rectangles of depth-ordered Gaussians [i0, i1) into the grid.
__device__ __forceinline__ void grid_add_rects(uint32_t* g, int w1, int tiles_x, int tiles_y,
                                               const uint32_t* __restrict__ packed, uint32_t i0, uint32_t i1) {
    constexpr int U = 8;  // loads in flight per thread
    for (uint32_t b = i0; b < i1; b += 256 * U) {
        uint32_t pk[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint32_t i = b + (uint32_t)(k * 256) + threadIdx.x;
            pk[k] = i < i1 ? packed[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (b + (uint32_t)(k * 256) + threadIdx.x < i1) grid_add_rect(g, w1, tiles_x, tiles_y, pk[k]);
    }
}

__device__ __forceinline__ uint32_t bin_valid(const Counters* cnt) { return cnt->overflow ? 0u : cnt->visible; }

// tile id -> (tx, ty) with the FP32 reciprocal of tiles_x, corrected to the
// exact quotient
__device__ __forceinline__ void tile_xy(uint32_t t, uint32_t tiles_x, float inv_tx, uint32_t* tx, uint32_t* ty) {
    uint32_t q = (uint32_t)((float)t * inv_tx);
    if (q * tiles_x > t) --q;
    if ((q + 1) * tiles_x <= t) ++q;
    *ty = q;
    *tx = t - q * tiles_x;
}

// Per block of BIN_BLOCK depth-ordered Gaussians: how many of their
// rectangles hold each tile, and the entry count of each of its rounds of
// 256 Gaussians.
__global__ __launch_bounds__(256) void k_bin_hist(const uint32_t* __restrict__ packed, const Counters* __restrict__ cnt,
                                                  int tiles_x, int tiles_y, uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ round_cnt, uint32_t* __restrict__ blk_tot) {
    static_assert(BIN_BLOCK == 8 * 256, "a block is eight rounds of 256");
    __shared__ uint32_t g[BIN_GRID_MAX];
    __shared__ uint32_t wsum[8][4];
    const uint32_t V = bin_valid(cnt);
    const uint32_t b0 = blockIdx.x * BIN_BLOCK;
    if (b0 >= V) return;  // uniform
    const int w1 = tiles_x + 1, h1 = tiles_y + 1;
    for (int c = threadIdx.x; c < w1 * h1; c += 256) g[c] = 0u;
    uint32_t pk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t i = b0 + (uint32_t)(k * 256) + threadIdx.x;
        pk[k] = i < V ? packed[i] : 0u;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool in = b0 + (uint32_t)(k * 256) + threadIdx.x < V;
        if (in) grid_add_rect(g, w1, tiles_x, tiles_y, pk[k]);
        const uint32_t ws = wave_sum(in ? rect_count(pk[k]) : 0u);
        if (lane == 0) wsum[k][w] = ws;
    }
    __syncthreads();
    const uint32_t nrounds = (V + 255) / 256;
    if (threadIdx.x < 8 && blockIdx.x * 8 + threadIdx.x < nrounds) {
        const int k = threadIdx.x;
        round_cnt[blockIdx.x * 8 + k] = wsum[k][0] + wsum[k][1] + wsum[k][2] + wsum[k][3];
    }
    if (threadIdx.x == 0) {  // the block's entries (its eight rounds)
        uint32_t b = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) b += wsum[k][0] + wsum[k][1] + wsum[k][2] + wsum[k][3];
        blk_tot[blockIdx.x] = b;
    }
    grid_prefix2d(g, w1, h1);
    const uint32_t n_tiles = (uint32_t)(tiles_x * tiles_y);
    const float inv_tx = 1.0f / (float)tiles_x;
    uint32_t* row = hist + (size_t)blockIdx.x * n_tiles;
    for (uint32_t t = threadIdx.x; t < n_tiles; t += 256) {
        uint32_t tx, ty;
        tile_xy(t, (uint32_t)tiles_x, inv_tx, &tx, &ty);
        row[t] = g[ty * w1 + tx];
    }
}

__device__ __forceinline__ void bin_groups(uint32_t V, uint32_t* nb, uint32_t* bpg) {
    *nb = (V + BIN_BLOCK - 1) / BIN_BLOCK;
    *bpg = (*nb + BIN_GROUPS - 1) / BIN_GROUPS;
}

// Per tile and group of consecutive blocks: the exclusive prefix of the
// block histograms inside the group (in place) and the group's total.
__global__ __launch_bounds__(256) void k_bin_prefix(uint32_t* __restrict__ hist, const Counters* __restrict__ cnt,
                                                    uint32_t n_tiles, uint32_t* __restrict__ gsum) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tiles) return;
    uint32_t nb, bpg;
    bin_groups(bin_valid(cnt), &nb, &bpg);
    const uint32_t b0 = blockIdx.y * bpg, b1 = min(nb, b0 + bpg);
    uint32_t run = 0;
    for (uint32_t b = b0; b < b1; b += 8) {
        uint32_t h[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = b + k < b1 ? hist[(size_t)(b + k) * n_tiles + t] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (b + k < b1) hist[(size_t)(b + k) * n_tiles + t] = run;
            run += h[k];
        }
    }
    gsum[blockIdx.y * n_tiles + t] = run;
}

// Per tile: the exclusive prefix of the group totals over groups (in place)
// and the tile's total, stored after the BIN_GROUPS group rows.
__global__ __launch_bounds__(256) void k_bin_groups(uint32_t* __restrict__ gsum, const Counters* __restrict__ cnt,
                                                    uint32_t n_tiles, uint32_t* __restrict__ tchunk) {
    __shared__ uint32_t red[4];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    const bool in = t < n_tiles;
    uint32_t nb, bpg;
    bin_groups(bin_valid(cnt), &nb, &bpg);
    const uint32_t ng = in && bpg ? (nb + bpg - 1) / bpg : 0u;
    uint32_t x[BIN_GROUPS];
#pragma unroll
    for (int g = 0; g < BIN_GROUPS; ++g) x[g] = (uint32_t)g < ng ? gsum[g * n_tiles + t] : 0u;
    uint32_t run = 0;
#pragma unroll
    for (int g = 0; g < BIN_GROUPS; ++g) {
        if ((uint32_t)g < ng) gsum[g * n_tiles + t] = run;
        run += x[g];
    }
    if (in) gsum[BIN_GROUPS * n_tiles + t] = run;
    // the 256 tiles' total, for the tile starts
    const uint32_t c = block_sum<256>(run, red);
    if (threadIdx.x == 0) tchunk[blockIdx.x] = c;
}

// Tile starts and round offsets, each in chunks of 256 (one workgroup per
// chunk, so that many compute units read the totals the previous kernels
// wrote): workgroups [0, ntc) take 256 tiles each, starting from the totals
// of the tile chunks before theirs, and store each tile's start (in the row
// after the totals) and range; the others take 256 rounds each, starting
// from the entry totals of the histogram blocks (eight rounds each) before
// theirs, and store each round's offset and, in start_round, the first round
// of every emission workgroup.  Workgroup 0 also copies the counters for the
// host (the frame's counters are final here).
__global__ __launch_bounds__(256) void k_bin_tiles(uint32_t* __restrict__ gsum, const Counters* __restrict__ cnt,
                                                   uint32_t n_tiles, uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ round_cnt,
                                                   uint32_t* __restrict__ round_off, uint32_t* __restrict__ start_round,
                                                   uint32_t nwg, Counters* host_cnt,
                                                   const uint32_t* __restrict__ tchunk,
                                                   const uint32_t* __restrict__ blk_tot) {
    __shared__ uint32_t red[4];
    __shared__ unsigned long long red64[4];
    if (blockIdx.x == 0 && threadIdx.x == 0) *host_cnt = *cnt;
    const uint32_t V = bin_valid(cnt);
    if (V == 0) return;  // uniform; the ranges were cleared
    const uint32_t ntc = (n_tiles + 255) / 256;
    if (blockIdx.x < ntc) {
        const uint32_t c = blockIdx.x;
        const uint32_t before = block_sum<256>(threadIdx.x < c ? tchunk[threadIdx.x] : 0u, red);
        const uint32_t t = c * 256 + threadIdx.x;
        const uint32_t tot = t < n_tiles ? gsum[(size_t)BIN_GROUPS * n_tiles + t] : 0u;
        uint32_t all;
        const uint32_t start = before + block_excl_scan<256>(tot, red, &all);
        if (t < n_tiles) {
            ranges[t] = tot ? make_uint2(start, start + tot) : make_uint2(0u, 0u);
            gsum[(size_t)(BIN_GROUPS + 1) * n_tiles + t] = start;
        }
        return;
    }
    const uint32_t k = blockIdx.x - ntc;
    const uint32_t nrounds = (V + 255) / 256;
    if (k * 256 >= nrounds) return;  // uniform
    uint64_t p = 0;
    for (uint32_t b = threadIdx.x; b < 32 * k; b += 256) p += blk_tot[b];
    const uint32_t before = (uint32_t)block_sum_u64(p, red64);
    const uint32_t r = k * 256 + threadIdx.x;
    const uint32_t x = r < nrounds ? round_cnt[r] : 0u;
    uint32_t all;
    const uint32_t o = before + block_excl_scan<256>(x, red, &all);
    if (r < nrounds) {
        round_off[r] = o;
        // workgroups whose first unit falls in round r's cost range
        const uint64_t c_lo = (uint64_t)o + (uint64_t)BIN_ROUND_COST * r;
        const uint64_t c_hi = (uint64_t)(o + x) + (uint64_t)BIN_ROUND_COST * (r + 1);
        for (uint64_t wk = (c_lo + BIN_PAIRS - 1) / BIN_PAIRS; wk < nwg && wk * BIN_PAIRS < c_hi; ++wk)
            start_round[wk] = r;
        if (r + 1 == nrounds) round_off[nrounds] = o + x;
    }
}

// Inclusive XOR prefix over the 64 lanes of a wave (same lane pattern as
// wave_incl_scan; lanes without a source see 0, the identity).
__device__ __forceinline__ uint32_t wave_incl_xor(uint32_t v) {
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Lane masks of one wave over the columns (or rows) 0..n-1: bit l of m[x] is
// set when lane l's interval [lo, hi] holds x.  Each lane toggles its bit at
// lo and at hi + 1 (m has n + 1 entries, cleared by the caller), and the XOR
// prefix over x leaves each bit set exactly inside its interval.
__device__ __forceinline__ void wave_interval_masks(unsigned long long* m, int n, bool valid, int lo, int hi) {
    const int lane = (int)(threadIdx.x & 63);
    if (valid) {
        atomicXor(&m[lo], 1ull << lane);
        atomicXor(&m[hi + 1], 1ull << lane);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t clo = 0, chi = 0;
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int x = c0 + lane;
        const unsigned long long v = x < n ? m[x] : 0ull;
        const uint32_t slo = wave_incl_xor((uint32_t)v) ^ clo, shi = wave_incl_xor((uint32_t)(v >> 32)) ^ chi;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (x < n) m[x] = ((unsigned long long)shi << 32) | slo;
        clo = readlane(slo, 63);
        chi = readlane(shi, 63);
    }
}

// Dense-first dispatch order of a frame's tiles for the blend: tiles by
// decreasing list length in 64 buckets of a quarter octave each (lengths up
// to 2^16 apart), so the longest lists start first and short ones fill the
// end of the launch instead of long ones running on after the rest are done.
// Within a bucket the order is whatever the atomics give: every tile's
// pixels are computed on their own, so the order changes only the timing.
// One workgroup of NT threads; hist: 64 words of LDS.
__device__ __forceinline__ uint32_t length_bucket(uint32_t n) {
    const uint32_t x = n + 1u;
    const int msb = 31 - __builtin_clz(x);
    const uint32_t frac = msb >= 2 ? (x >> (msb - 2)) & 3u : (x << (2 - msb)) & 3u;
    return 63u - min(63u, 4u * (uint32_t)msb + frac);
}
template <int NT>
__device__ void tile_order(const uint2* __restrict__ ranges, uint32_t n_tiles, uint32_t* __restrict__ order,
                           uint32_t* hist) {
    for (int i = (int)threadIdx.x; i < 64; i += NT) hist[i] = 0u;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n_tiles; t += NT) {
        const uint2 r = ranges[t];
        atomicAdd(&hist[length_bucket(r.y - r.x)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < 64; ++b) {
            const uint32_t c = hist[b];
            hist[b] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n_tiles; t += NT) {
        const uint2 r = ranges[t];
        order[atomicAdd(&hist[length_bucket(r.y - r.x)], 1u)] = t;
    }
}

// The same as a launch of its own, for frames whose ranges come from k_ranges.
__global__ __launch_bounds__(256) void k_tile_order(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                    uint32_t* __restrict__ order) {
    __shared__ uint32_t hist[64];
    tile_order<256>(ranges, n_tiles, order, hist);
}

// Writes the entries of the depth-first emission order (Gaussians in depth
// order, tiles row-major over each rectangle) to their sorted positions:
// record ids, and with DEBUG also each entry's tile id and depth word; each
// workgroup takes BIN_PAIRS units of work.  cntr holds, per tile, the
// position of its next entry; inside a round each entry adds the count of
// earlier Gaussians of the round that hold its tile (the waves' column and
// row lane masks), and the round's last Gaussian holding a tile moves that
// tile's position.  Workgroup 0 writes the blend's dispatch order from the
// (final) ranges instead, when `order` is given; the others take the
// emission work.
template <bool DEBUG>
__global__ __launch_bounds__(256) void k_bin_emit(const uint2* __restrict__ ranges, uint32_t* __restrict__ order,
                                                  const uint32_t* __restrict__ sorted_rec,
                                                  const uint32_t* __restrict__ packed, const Counters* __restrict__ cnt,
                                                  const uint32_t* __restrict__ hist, const uint32_t* __restrict__ gsum,
                                                  const uint32_t* __restrict__ round_off,
                                                  const uint32_t* __restrict__ start_round, int tiles_x, int tiles_y,
                                                  uint32_t* __restrict__ val_out, uint32_t* __restrict__ tile_out,
                                                  uint32_t* __restrict__ depth_out,
                                                  const uint32_t* __restrict__ zkey) {
    // dynamic LDS sized for the view's grid: column and row lane masks per
    // wave (one spare entry each for the interval ends), next position per cell
    extern __shared__ __align__(16) unsigned char bin_smem[];
    unsigned long long* colm = reinterpret_cast<unsigned long long*>(bin_smem);  // [4][tiles_x + 1]
    unsigned long long* rowm = colm + 4 * (tiles_x + 1);                         // [4][tiles_y + 1]
    uint32_t* cntr = reinterpret_cast<uint32_t*>(rowm + 4 * (tiles_y + 1));
    __shared__ uint32_t red[4], wmax[4], pick;
    __shared__ uint32_t pre[257], own[256], srec[256], spk[256];
    __shared__ float sinv[256];
    if (blockIdx.x == 0) {  // uniform
        if (order) tile_order<256>(ranges, (uint32_t)(tiles_x * tiles_y), order, pre);
        return;
    }
    const int bid = (int)blockIdx.x - 1;  // the emission workgroup
    const uint32_t V = bin_valid(cnt);
    const uint32_t D = cnt->D;
    if (V == 0) return;  // uniform
    // Work is split by cost: a round of 256 Gaussians costs its entries plus
    // BIN_ROUND_COST (its fixed steps), so round r starts at cost
    // C(r) = round_off[r] + BIN_ROUND_COST r; its first BIN_ROUND_COST units
    // stand for the fixed steps, the rest for its entries in order.
    const uint32_t nrounds = (V + 255) / 256;
    const uint64_t total_cost = (uint64_t)round_off[nrounds] + (uint64_t)BIN_ROUND_COST * nrounds;
    const uint32_t nact = (uint32_t)((total_cost + BIN_PAIRS - 1) / BIN_PAIRS);
    if ((uint32_t)bid >= nact) return;  // uniform
    // XCD x takes a contiguous run of the cost ranges in use: the entries
    // neighbouring workgroups write to one tile's list are adjacent and meet
    // in one L2
    const uint64_t A = (uint64_t)xcd_segment(bid, (int)nact) * BIN_PAIRS;
    const uint64_t B = min(total_cost, A + BIN_PAIRS);
    auto cost = [&](uint32_t r) -> uint64_t { return (uint64_t)round_off[r] + (uint64_t)BIN_ROUND_COST * r; };
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // the round holding cost A (the last r with C(r) <= A)
    const uint32_t R = start_round[A / BIN_PAIRS];
    // entered part way (past its fixed steps and first entries), round R is
    // counted into the start positions and its entries step back by their
    // tile's count in the round
    const bool part = A > cost(R) + BIN_ROUND_COST;
    const uint32_t cb = R * 256 / BIN_BLOCK;
    uint32_t nb, bpg;
    bin_groups(V, &nb, &bpg);
    const uint32_t grp = cb / bpg;
    const int w1 = tiles_x + 1, h1 = tiles_y + 1, ncell = w1 * h1;
    const uint32_t n_tiles = (uint32_t)(tiles_x * tiles_y);
    const float inv_tx = 1.0f / (float)tiles_x;
    // next positions at the start of round R (of R + 1 when entered part
    // way): tile starts, block prefixes, and the block's Gaussians before
    for (int c = threadIdx.x; c < ncell; c += 256) cntr[c] = 0u;
    __syncthreads();
    grid_add_rects(cntr, w1, tiles_x, tiles_y, packed, cb * BIN_BLOCK, part ? min(V, R * 256 + 256) : R * 256);
    __syncthreads();
    grid_prefix2d(cntr, w1, h1);
    {
        const uint32_t* hrow = hist + (size_t)cb * n_tiles;
        const uint32_t* grow = gsum + (size_t)grp * n_tiles;
        const uint32_t* srow = gsum + (size_t)(BIN_GROUPS + 1) * n_tiles;
        constexpr int U = 8;
        for (uint32_t t0 = 0; t0 < n_tiles; t0 += 256 * U) {
            uint32_t h[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t t = t0 + (uint32_t)(k * 256) + threadIdx.x;
                h[k] = t < n_tiles ? hrow[t] + grow[t] + srow[t] : 0u;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t t = t0 + (uint32_t)(k * 256) + threadIdx.x;
                if (t < n_tiles) {
                    uint32_t tx, ty;
                    tile_xy(t, (uint32_t)tiles_x, inv_tx, &tx, &ty);
                    cntr[ty * w1 + tx] += h[k];
                }
            }
        }
    }
    __syncthreads();
    unsigned long long* cw = colm + w * (tiles_x + 1);
    unsigned long long* rw = rowm + w * (tiles_y + 1);
    // each round loads the next one's Gaussians ahead
    uint32_t nx_rec = 0, nx_p = 0;
    if (R * 256 + threadIdx.x < V) {
        nx_rec = sorted_rec[R * 256 + threadIdx.x];
        nx_p = packed[R * 256 + threadIdx.x];
    }
    for (uint32_t r = R; r < nrounds; ++r) {
        const uint64_t cr = cost(r);
        if (cr >= B) break;  // uniform
        const uint32_t i = r * 256 + threadIdx.x;
        const bool valid = i < V;
        const uint32_t rec = nx_rec, p = nx_p;
        if (i + 256 < V) {
            nx_rec = sorted_rec[i + 256];
            nx_p = packed[i + 256];
        }
        uint32_t n = 0;
        int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
        if (valid) {
            x0 = (int)(p & 0xffu);
            y0 = (int)((p >> 8) & 0xffu);
            x1 = (int)((p >> 16) & 0xffu);
            y1 = (int)(p >> 24);
            n = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
        }
        // this wave's column and row lane masks
        for (int x = lane; x <= tiles_x; x += 64) cw[x] = 0ull;
        for (int y = lane; y <= tiles_y; y += 64) rw[y] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        wave_interval_masks(cw, tiles_x, valid, x0, x1);
        wave_interval_masks(rw, tiles_y, valid, y0, y1);
        uint32_t tot;
        const uint32_t ex = block_excl_scan<256>(n, red, &tot);
        // this workgroup's slots of the round: [js, je)
        const uint64_t c0 = cr + BIN_ROUND_COST;
        const uint32_t js = (uint32_t)min((uint64_t)tot, A > c0 ? A - c0 : 0ull);
        const uint32_t je = (uint32_t)min((uint64_t)tot, B > c0 ? B - c0 : 0ull);
        const bool first_part = part && r == R;
        const uint32_t wstart = js & ~255u;
        pre[threadIdx.x + 1] = ex + n;
        if (threadIdx.x == 0) {
            pre[0] = 0;
            pick = 0u;
        }
        own[threadIdx.x] = 0u;
        srec[threadIdx.x] = rec;
        spk[threadIdx.x] = p;
        sinv[threadIdx.x] = valid ? 1.0f / (float)(x1 - x0 + 1) : 0.0f;
        __syncthreads();
        // owner of the slot before the first window: the last Gaussian whose
        // first slot precedes it
        if (wstart > 0 && n && ex < wstart) atomicMax(&pick, threadIdx.x);
        __syncthreads();
        uint32_t carry = pick;
        // a move of a next position found in a window is applied once every
        // read of that window is done (after the next barrier)
        int pend_cell = -1;
        uint32_t pend_val = 0;
        // windows of 256 slots: a slot's owner is the last Gaussian whose
        // first slot is at or before it (round-tagged marks and a prefix
        // maximum, as in k_duplicate)
        for (uint32_t j0 = wstart, m = wstart >> 8; j0 < je; j0 += 256, ++m) {
            if (n && (ex >> 8) == m) own[ex & 255u] = (m << 8) | threadIdx.x;
            __syncthreads();
            if (pend_cell >= 0) {
                cntr[pend_cell] += pend_val;
                pend_cell = -1;
            }
            const uint32_t incl = wave_incl_max(own[threadIdx.x]);
            if (lane == 63) wmax[w] = incl;
            __syncthreads();
            uint32_t o = max(incl, (m << 8) | carry), all = (m << 8) | carry;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t xw = wmax[v];
                if (v < w) o = max(o, xw);
                all = max(all, xw);
            }
            carry = all & 0xffu;
            const uint32_t j = j0 + threadIdx.x;
            if (j >= js && j < je) {
                const uint32_t eo = o & 0xffu;
                const uint32_t k = j - pre[eo];
                const uint32_t pk = spk[eo];
                const uint32_t ex0 = pk & 0xffu, ey0 = (pk >> 8) & 0xffu;
                const uint32_t nx = ((pk >> 16) & 0xffu) - ex0 + 1u;
                // k / nx through the FP32 reciprocal, corrected to the exact quotient
                uint32_t qq = (uint32_t)((float)k * sinv[eo]);
                if (qq * nx > k) --qq;
                if ((qq + 1) * nx <= k) ++qq;
                const int ty = (int)(ey0 + qq), tx = (int)(ex0 + (k - qq * nx));
                const int we = (int)(eo >> 6), le = (int)(eo & 63u);
                const unsigned long long below = le == 0 ? 0ull : (~0ull >> (64 - le));
                uint32_t before = 0, total = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const unsigned long long mm = colm[v * (tiles_x + 1) + tx] & rowm[v * (tiles_y + 1) + ty];
                    const uint32_t c = (uint32_t)__builtin_popcountll(mm);
                    total += c;
                    if (v < we) before += c;
                    else if (v == we) before += (uint32_t)__builtin_popcountll(mm & below);
                }
                const int cell = ty * w1 + tx;
                const uint32_t pos = cntr[cell] + before - (first_part ? total : 0u);
                if (pos < D) {
                    const uint32_t rr = srec[eo];
                    val_out[pos] = rr;
                    if (DEBUG) {
                        tile_out[pos] = (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)tx;
                        depth_out[pos] = zkey[rr];
                    }
                }
                // the round's last Gaussian holding the tile: no later slot
                // of the round reads its position
                if (!first_part && before + 1u == total) {
                    pend_cell = cell;
                    pend_val = total;
                }
            }
        }
        __syncthreads();
        if (pend_cell >= 0) cntr[pend_cell] += pend_val;
        if (je < tot) break;  // uniform: the range ends inside this round
        __syncthreads();
    }
}

// ------------------------------------------------------------------- blend

constexpr float ALPHA_MAX = 0.99f;
constexpr float T_MIN = 1e-4f;

__device__ __forceinline__ uint8_t to_u8(float x) {
    return (uint8_t)floorf(__builtin_fmaf(fminf(fmaxf(x, 0.0f), 1.0f), 255.0f, 0.5f));
}

struct BlendArgs {
    const ViewParams* views;
    int nviews;
    uint32_t n_tiles;
    const uint2* ranges;
    const uint32_t* vals;
    const Rec* rec;
    uint32_t nrec;
    unsigned long long* work;
    int cull;  // drop entries below the skip threshold on the whole block (never changes a pixel)
    const uint32_t* order;  // dense-first dispatch order of the tiles (null: XCD chunks)
};

// Per-wave LDS slice of staged Gaussians: block-relative centre (u, v of the
// first 8x8 block; v of the second one when a lane owns two pixels), the
// exponent coefficients and the colour.
template <int BD>
struct Stage {
    float4 a[64 * BD];  // u_rel, A, r, g   (what the per-pair loop reads)
    float4 b[64 * BD];  // v_rel0, B, C, L (what the row terms read)
    float2 c[64 * BD];  // b, v_rel1
};


// Does the Gaussian with exponent e(d) = A dx^2 + B dx dy + C dy^2 + L
// (negative-definite quadratic part) stay below the skip threshold on the
// whole rectangle [dx0, dx1] x [dy0, dy1] of offsets?  The maximum of a
// concave quadratic over a rectangle is at the unconstrained maximum when
// that lies inside, else on an edge facing the centre, where it is a 1D
// concave quadratic maximised at a clamped stationary point.  The test is
// conservative: it answers yes only with a margin far above the FP32
// rounding of this bound and of the per-pixel exponent, so a Gaussian it
// removes would have been skipped at every pixel of the rectangle.
__device__ __forceinline__ bool below_threshold(float A, float B, float C, float L, float dx0, float dx1, float dy0,
                                                float dy1) {
    if (!(A < 0.0f && C < 0.0f && B * B < 4.0f * A * C)) return false;  // not concave: keep it
    float q = 0.0f;
    if (!(dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f)) {
        const float ra = __builtin_amdgcn_rcpf(2.0f * A), rc = __builtin_amdgcn_rcpf(2.0f * C);
        auto edge_x = [&](float cx) {  // dx = cx fixed, best dy
            const float dy = fminf(fmaxf(-B * cx * rc, dy0), dy1);
            return (A * cx + B * dy) * cx + C * dy * dy;
        };
        auto edge_y = [&](float cy) {  // dy = cy fixed, best dx
            const float dx = fminf(fmaxf(-B * cy * ra, dx0), dx1);
            return (C * cy + B * dx) * cy + A * dx * dx;
        };
        // the maximum lies on a face visible from the centre (visibility is
        // affine-invariant, so it holds in the quadratic's own metric): the
        // x-face and the y-face on the centre's side suffice
        q = fmaxf(edge_x(dx1 < 0.0f ? dx1 : dx0), edge_y(dy1 < 0.0f ? dy1 : dy0));
    }
    const float r2 = fmaxf(dx0 * dx0, dx1 * dx1) + fmaxf(dy0 * dy0, dy1 * dy1);
    const float margin = 0.02f + 1e-5f * (fabsf(A) + fabsf(B) + fabsf(C)) * r2;
    return q + L < LOG2_ALPHA_MIN - margin;  // false for NaN
}

// One tile of TW x TH pixels.  Each wave owns a block of 8 x (8 PPL) pixels
// (PPL pixels per lane, one per stacked 8x8 sub-block); wave w takes block
// (w mod TW/8, w div TW/8).  The wave walks the tile's depth-sorted list in
// batches of 64 * BD entries: every lane fetches entries, keeps those whose
// pixel box meets the wave's block (and, with culling on, whose exponent can
// reach the skip threshold somewhere on it), compacts them into the wave's
// LDS slice (ballot + mbcnt) and the 64 lanes then composite them front to
// back.  Each pixel's operations (and their rounding) are the same for every
// tile shape and PPL: offsets are taken from the 8x8 sub-block's own origin,
// and the entries culling drops are ones every pixel of the block skips.  A wave
// leaves as soon as all of its pixels have terminated; there is no barrier
// between the waves of a tile.
template <int TW, int TH, int BD, int PPL, bool COUNT>
__device__ __forceinline__ void blend_tile(const BlendArgs& A, uint32_t tile, int w, Stage<BD>& S) {
    constexpr int BX = TW / 8;
    constexpr int BATCH = 64 * BD;
    int vi = 0;
    {
        int lo = 0, hi = A.nviews - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
        }
        vi = lo;
    }
    const ViewParams& v = A.views[vi];
    const uint32_t lt = tile - v.tile_base;
    const int tx = (int)(lt % (uint32_t)v.tiles_x), ty = (int)(lt / (uint32_t)v.tiles_x);
    const int lane = threadIdx.x & 63;
    const int sx = tx * TW + (w % BX) * 8, sy = ty * TH + (w / BX) * 8 * PPL;
    const int px = sx + (lane & 7);
    const float pxr = (float)(lane & 7) + 0.5f, pyr = (float)(lane >> 3) + 0.5f;
    const float fsx = (float)sx;
    float fsy[PPL];
    int py[PPL];
    bool done[PPL];
    float T[PPL], cr[PPL], cg[PPL], cb[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        fsy[p] = (float)(sy + 8 * p);
        py[p] = sy + 8 * p + (lane >> 3);
        done[p] = !(px < v.width && py[p] < v.height);
        T[p] = 1.0f;
        cr[p] = cg[p] = cb[p] = 0.0f;
    }
    const uint2 rg = A.ranges[tile];
    uint32_t n_eval = 0, n_contrib = 0;  // (pixel, Gaussian) evaluations / contributions, COUNT only
    // the wave's block clipped to the image: the only pixels it must cover
    const int bx1 = min(sx + 7, v.width - 1), by1 = min(sy + 8 * PPL - 1, v.height - 1);

    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
        bool alive = false;
#pragma unroll
        for (int p = 0; p < PPL; ++p) alive = alive || !done[p];
        if (ballot(alive) == 0) break;
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < BD; ++k) {
            const uint32_t i = base + (uint32_t)(k * 64 + lane);
            bool hit = false;
            uint32_t r = 0;
            if (i < rg.y) r = A.vals[i];
            if (i < rg.y && r < A.nrec) {
                const uint2 b = A.rec[r].bbox;
                const int x0 = (int)(b.x & 0xffffu), y0 = (int)(b.x >> 16);
                const int x1 = (int)(b.y & 0xffffu), y1 = (int)(b.y >> 16);
                hit = !(x1 < sx || x0 > bx1 || y1 < sy || y0 > by1);
            }
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b1 = a, c2 = a;
            float u = 0.f, v0 = 0.f;
            if (hit) {
                a = A.rec[r].r0;
                b1 = A.rec[r].r1;
                c2 = A.rec[r].r2;
                // pixel centre relative to each 8x8 sub-block origin, hi and lo parts combined here
                u = (a.x - fsx) + a.z;
                v0 = (a.y - fsy[0]) + a.w;
                hit = !(A.cull && below_threshold(b1.x, b1.y, b1.z, b1.w, 0.5f - u, 7.5f - u, 0.5f - v0,
                                                  (float)(8 * PPL) - 0.5f - v0));
            }
            const uint64_t m = ballot(hit);
            if (hit) {
                const uint32_t slot = cnt + bits_below(m);
                S.a[slot] = make_float4(u, b1.x, c2.x, c2.y);
                S.b[slot] = make_float4(v0, b1.y, b1.z, b1.w);
                S.c[slot] = make_float2(c2.z, PPL > 1 ? (a.y - fsy[PPL - 1]) + a.w : 0.0f);
            }
            cnt += (uint32_t)__builtin_popcountll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (PPL == 1) {
            // Eight entries at a time.  Lane l forms, for entry j0 + l/8 and
            // pixel row l mod 8, the row terms B dy and C dy^2 + L (the very
            // products and sums of the per-pixel exponent, so every pixel's
            // arithmetic is unchanged); the lanes of a row then fetch theirs
            // with a cross-lane permute, which leaves dx and two FMAs per
            // (pixel, Gaussian) pair.  The permutes run on every lane.
            const float yrow = (float)(lane & 7) + 0.5f;
            for (uint32_t j0 = 0; j0 < cnt; j0 += 8) {
                // the pixels still compositing, as a wave mask: the per-pair
                // decisions are combined in scalar registers and applied
                // with one select each
                uint64_t live = ballot(!done[0]);
                if (live == 0) break;
                const uint32_t jg = min(j0 + (uint32_t)(lane >> 3), cnt - 1);
                const float4 gb = S.b[jg];
                const float dyg = yrow - gb.x;
                const float pg = gb.y * dyg;
                const float qg = __builtin_fmaf(gb.z * dyg, dyg, gb.w);
                const uint32_t nk = min(8u, cnt - j0);
                auto pair = [&](uint32_t k) {
                    const int src = (int)(k * 8) + (lane >> 3);
                    const float P = __shfl(pg, src, 64);
                    const float Q = __shfl(qg, src, 64);
                    // straight-line update (no branches per pair): a pixel
                    // that is done, or an alpha below the threshold, or a
                    // stop, leaves the colour and T exactly as they are
                    const float4 ua = S.a[j0 + k];
                    const float cz = S.c[j0 + k].x;
                    const float dx = pxr - ua.x;
                    const float e = __builtin_fmaf(__builtin_fmaf(ua.y, dx, P), dx, Q);
                    const float alpha = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(e));
                    const float t0 = T[0];
                    const float at = alpha * t0;
                    const float tn = t0 - at;
                    const uint64_t use = ballot(alpha >= ALPHA_MIN) & live;
                    const uint64_t stop = use & ballot(tn < T_MIN);
                    const bool acc = __builtin_amdgcn_inverse_ballot_w64(use & ~stop);
                    if (COUNT) {
                        n_eval += __builtin_amdgcn_inverse_ballot_w64(live) ? 1u : 0u;
                        n_contrib += acc ? 1u : 0u;
                    }
                    live &= ~stop;
                    // a weight of zero leaves the (finite) colour sums exactly
                    // as they are, with one select instead of three
                    const float wgt = acc ? at : 0.0f;
                    cr[0] = __builtin_fmaf(wgt, ua.z, cr[0]);
                    cg[0] = __builtin_fmaf(wgt, ua.w, cg[0]);
                    cb[0] = __builtin_fmaf(wgt, cz, cb[0]);
                    T[0] = acc ? tn : t0;
                };
                if (nk == 8) {
                    // a full group: no branch between the pairs, so the
                    // LDS reads of later pairs are issued ahead
#pragma unroll
                    for (uint32_t k = 0; k < 8; ++k) pair(k);
                } else {
#pragma unroll
                    for (uint32_t k = 0; k < 8; ++k) {
                        if (k >= nk) break;
                        pair(k);
                    }
                }
                done[0] = !__builtin_amdgcn_inverse_ballot_w64(live);
            }
        } else if (alive) {
            for (uint32_t j = 0; j < cnt; ++j) {
                const float4 a = S.a[j];
                const float4 b = S.b[j];
                const float2 c = S.c[j];
                const float dx = pxr - a.x;
                bool all_done = true;
#pragma unroll
                for (int p = 0; p < PPL; ++p) {
                    const float vrel = p == 0 ? b.x : c.y;
                    const float dy = pyr - vrel;
                    const float e = __builtin_fmaf(__builtin_fmaf(a.y, dx, b.y * dy), dx,
                                                   __builtin_fmaf(b.z * dy, dy, b.w));
                    const float alpha = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(e));
                    if (!done[p]) {
                        if (COUNT) ++n_eval;
                        if (alpha >= ALPHA_MIN) {
                            const float wgt = alpha * T[p];
                            const float Tn = T[p] - wgt;
                            if (Tn < T_MIN) {
                                done[p] = true;
                            } else {
                                cr[p] = __builtin_fmaf(wgt, a.z, cr[p]);
                                cg[p] = __builtin_fmaf(wgt, a.w, cg[p]);
                                cb[p] = __builtin_fmaf(wgt, c.x, cb[p]);
                                T[p] = Tn;
                                if (COUNT) ++n_contrib;
                            }
                        }
                    }
                    all_done = all_done && done[p];
                }
                if (all_done) break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (COUNT) {
        const uint32_t se = wave_sum(n_eval), sc = wave_sum(n_contrib);
        if (lane == 0) {
            atomicAdd(&A.work[0], (unsigned long long)se);
            atomicAdd(&A.work[1], (unsigned long long)sc);
        }
    }
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        if (px < v.width && py[p] < v.height) {
            const float r = __builtin_fmaf(T[p], v.bg[0], cr[p]);
            const float g = __builtin_fmaf(T[p], v.bg[1], cg[p]);
            const float b = __builtin_fmaf(T[p], v.bg[2], cb[p]);
            const size_t pix = (size_t)py[p] * (size_t)v.width + (size_t)px;
            if (v.fmt == 1) {
                float* out = reinterpret_cast<float*>(v.out_ptr) + pix * 3;
                out[0] = r;
                out[1] = g;
                out[2] = b;
            } else {
                uint8_t* out = reinterpret_cast<uint8_t*>(v.out_ptr) + pix * 3;
                out[0] = to_u8(r);
                out[1] = to_u8(g);
                out[2] = to_u8(b);
            }
        }
    }
}

// One workgroup per tile, in the dense-first order when one is given (the
// longest lists first: the launch ends with short tiles instead of a tail of
// long ones).  Otherwise XCD-aware: consecutive workgroup ids go round-robin
// to the 8 XCDs; XCD x takes the chunks of BLEND_CHUNK consecutive tiles
// numbered x, x + 8, x + 16, ..., so neighbouring tiles (which share
// Gaussians) meet in the same L2 while every XCD gets a share of every part
// of the image (dense and sparse regions alike).
constexpr uint32_t BLEND_CHUNK = 16;
template <int TW, int TH, int BD, int PPL, bool COUNT>
__global__ __launch_bounds__(TW* TH / PPL) void k_blend(BlendArgs A) {
    constexpr int NW = TW * TH / (64 * PPL);
    __shared__ Stage<BD> stage[NW];
    uint32_t tile;
    if (A.order) {
        if (blockIdx.x >= A.n_tiles) return;
        tile = A.order[blockIdx.x];
    } else {
        const uint32_t j = blockIdx.x >> 3, x = blockIdx.x & 7;
        tile = ((j / BLEND_CHUNK) * 8u + x) * BLEND_CHUNK + (j % BLEND_CHUNK);
        if (tile >= A.n_tiles) return;
    }
    blend_tile<TW, TH, BD, PPL, COUNT>(A, tile, threadIdx.x >> 6, stage[threadIdx.x >> 6]);
}

// Persistent form for many views of uneven size: a fixed grid of resident
// workgroups pulls tiles from 8 device work queues, one per band of
// consecutive tiles; a workgroup starts on the band of its XCD (id mod 8) and
// moves on to the other bands when its own is drained.  The queue counters are
// cleared by k_scan_visible each frame; every workgroup exits once all bands
// are drained.
template <int TW, int TH, int BD, int PPL>
__global__ __launch_bounds__(TW* TH / PPL) void k_blend_persistent(BlendArgs A, uint32_t* __restrict__ queue) {
    constexpr int NW = TW * TH / (64 * PPL);
    __shared__ Stage<BD> stage[NW];
    __shared__ uint32_t next;
    const uint32_t per = (A.n_tiles + 7) / 8;
    const int home = blockIdx.x & 7;
    for (int k = 0; k < 8; ++k) {
        const int band = (home + k) & 7;
        const uint32_t first = (uint32_t)band * per;
        const uint32_t band_end = min(A.n_tiles, first + per);
        if (first >= band_end) continue;
        for (;;) {
            if (threadIdx.x == 0) next = first + atomicAdd(&queue[band], 1u);
            __syncthreads();
            const uint32_t tile = next;
            __syncthreads();
            if (tile >= band_end) break;
            blend_tile<TW, TH, BD, PPL, false>(A, tile, threadIdx.x >> 6, stage[threadIdx.x >> 6]);
        }
    }
}

// One view's parameters, passed by value as a kernel argument, stored to
// device memory (the allocation-free entry point has no pinned host copy).
__global__ void k_store_view(ViewParams v, ViewParams* __restrict__ dst) {
    constexpr int W = (int)(sizeof(ViewParams) / 4);
    static_assert(sizeof(ViewParams) % 4 == 0, "view parameters are whole words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
    for (int i = threadIdx.x; i < W; i += blockDim.x) reinterpret_cast<uint32_t*>(dst)[i] = src[i];
}

// Fill of n words (clears the counter block the allocation-free entry point
// keeps in its fixed scratch array).
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t value) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = value;
}

__global__ void k_wave_scan_selftest(const uint32_t* in, uint32_t* out, int n) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const uint32_t x = i < n ? in[i] : 0u;
    const uint32_t s = wave_incl_scan(x);
    if (i < n) out[i] = s;
}

// ------------------------------------------------------------- launchers

#define TIGAS_LAUNCH_SHM(kernel, grid, block, shm, st, ...)                               \
    do {                                                                                  \
        KernelTimer* kt_ = g_kernel_timer;                                                \
        if (kt_) kt_->before(reinterpret_cast<const void*>(kernel), st);                 \
        hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                    \
        if (kt_) kt_->after(st);                                                          \
    } while (0)
#define TIGAS_LAUNCH(kernel, grid, block, st, ...) TIGAS_LAUNCH_SHM(kernel, grid, block, 0, st, __VA_ARGS__)

template <int ST>
static void preprocess_deg(int deg, dim3 grid, const SceneView& s, const ViewParams* v, int nv, uint32_t rb,
                           uint32_t np, uint32_t vb, const PreOut& o, hipStream_t st) {
    switch (deg) {
        case 0: TIGAS_LAUNCH((k_preprocess<ST, 0>), grid, dim3(K1_THREADS), st, s, v, nv, rb, np, vb, o); break;
        case 1: TIGAS_LAUNCH((k_preprocess<ST, 1>), grid, dim3(K1_THREADS), st, s, v, nv, rb, np, vb, o); break;
        case 2: TIGAS_LAUNCH((k_preprocess<ST, 2>), grid, dim3(K1_THREADS), st, s, v, nv, rb, np, vb, o); break;
        default: TIGAS_LAUNCH((k_preprocess<ST, 3>), grid, dim3(K1_THREADS), st, s, v, nv, rb, np, vb, o); break;
    }
}

void launch_preprocess(const SceneView& s, const ViewParams* views_dev, const ViewParams* views_host, int nviews,
                       uint32_t rec_base, uint32_t n_pad, uint32_t view_base, const PreOut& o, hipStream_t st) {
    // the SH coefficients loaded are those of the highest degree any view uses
    int deg = 0;
    for (int i = 0; i < nviews; ++i) deg = views_host[i].sh_degree > deg ? views_host[i].sh_degree : deg;
    const dim3 grid(n_pad / K1_THREADS);
    if (s.storage == 0) preprocess_deg<0>(deg, grid, s, views_dev, nviews, rec_base, n_pad, view_base, o, st);
    else if (s.storage == 1) preprocess_deg<1>(deg, grid, s, views_dev, nviews, rec_base, n_pad, view_base, o, st);
    else preprocess_deg<2>(deg, grid, s, views_dev, nviews, rec_base, n_pad, view_base, o, st);
}


void launch_store_view(const ViewParams& v, ViewParams* dst, hipStream_t st) {
    TIGAS_LAUNCH(k_store_view, dim3(1), dim3(64), st, v, dst);
}

void launch_fill_u32(uint32_t* p, uint32_t n, uint32_t value, hipStream_t st) {
    if (n == 0) return;
    TIGAS_LAUNCH(k_fill_u32, dim3(std::min<uint32_t>(1024u, (n + 255) / 256)), dim3(256), st, p, n, value);
}

void launch_scan_visible(const PreOut& o, int nblk, uint32_t* blk_off, Counters* cnt, uint32_t cap,
                         const ZeroList& zl, hipStream_t st) {
    const int nchunks = std::max(1, (nblk + SCAN_CHUNK - 1) / SCAN_CHUNK);
    TIGAS_LAUNCH(k_chunk_totals, dim3(nchunks), dim3(SCAN_THREADS), st, (const uint32_t*)o.blk_vis, nblk,
                 (const uint32_t*)o.blk_sum, (const uint32_t*)o.blk_fb, o.chunk_vis, o.chunk_dup, o.chunk_fb);
    TIGAS_LAUNCH(k_scan_visible, dim3(nchunks), dim3(SCAN_THREADS), st, (const uint32_t*)o.blk_vis, nblk,
                 (const uint32_t*)o.chunk_vis, (const unsigned long long*)o.chunk_dup, (const uint32_t*)o.chunk_fb,
                 nchunks, blk_off, cnt, cap, zl);
}

void launch_compact(const PreOut& o, int nblk, const uint32_t* blk_off, uint32_t* key, uint32_t* val, uint32_t* ext,
                    const ViewParams* views_dev, hipStream_t st) {
    if (nblk == 0) return;
    TIGAS_LAUNCH(k_compact, dim3((nblk + 3) / 4), dim3(K1_THREADS), st, o.zkey, (const uint2*)o.rect,
                 blk_off, nblk, key, val, ext, (const Counters*)o.cnt, (const uint2*)o.fb_list, o.fb_cap, views_dev,
                 (const uint32_t*)o.blk_view, o.rec);
}

void launch_duplicate(const PreOut& o, int nblk, const uint32_t* sorted_rec, const uint2* sorted_rect,
                      const uint32_t* sorted_packed,
                      uint32_t* blk_sum2, uint32_t* blk_off2, const Counters* cnt, uint32_t cap,
                      const ViewParams* views_dev, uint32_t* tile_out, uint32_t* val_out, uint32_t* depth_out,
                      hipStream_t st) {
    if (nblk == 0) return;
    TIGAS_LAUNCH(k_sorted_sums, dim3(std::min(nblk, 8192)), dim3(K1_THREADS), st, sorted_rect, sorted_packed, cnt, nblk,
                 blk_sum2);
    const int nchunks = std::max(1, (nblk + SCAN_CHUNK - 1) / SCAN_CHUNK);
    TIGAS_LAUNCH(k_chunk_totals, dim3(nchunks), dim3(SCAN_THREADS), st, (const uint32_t*)blk_sum2, nblk,
                 (const uint32_t*)nullptr, (const uint32_t*)nullptr, o.chunk_dups, (unsigned long long*)nullptr,
                 (uint32_t*)nullptr);
    TIGAS_LAUNCH(k_scan_dups, dim3(nchunks), dim3(SCAN_THREADS), st, (const uint32_t*)blk_sum2, nblk,
                 (const uint32_t*)o.chunk_dups, blk_off2, nchunks, (Counters*)nullptr);
    if (depth_out)
        TIGAS_LAUNCH(k_duplicate<true>, dim3(nblk), dim3(K1_THREADS), st, sorted_rec, sorted_rect, sorted_packed,
                     o.zkey, (const uint32_t*)blk_off2, o.blk_view, cnt, cap, views_dev, tile_out, val_out, depth_out);
    else
        TIGAS_LAUNCH(k_duplicate<false>, dim3(nblk), dim3(K1_THREADS), st, sorted_rec, sorted_rect, sorted_packed,
                     o.zkey, (const uint32_t*)blk_off2, o.blk_view, cnt, cap, views_dev, tile_out, val_out, depth_out);
}

void launch_duplicate_culled(const PreOut& o, int nblk, const uint32_t* sorted_rec, const uint32_t* sorted_packed,
                             uint32_t* blk_cnt, uint32_t* blk_off, Counters* cnt, const ViewParams* views_dev,
                             int tile_w, int tile_h, uint32_t* tile_out, uint32_t* val_out, uint32_t* depth_out,
                             hipStream_t st) {
    if (nblk == 0) return;
    TIGAS_LAUNCH((k_duplicate_culled<true, false>), dim3(nblk), dim3(K1_THREADS), st, sorted_rec, sorted_packed,
                 o.zkey, (const uint32_t*)nullptr, blk_cnt, (const uint32_t*)o.blk_view, (const Counters*)cnt,
                 views_dev, (const Rec*)o.rec, tile_w, tile_h, (uint32_t*)nullptr, (uint32_t*)nullptr,
                 (uint32_t*)nullptr);
    const int nchunks = std::max(1, (nblk + SCAN_CHUNK - 1) / SCAN_CHUNK);
    TIGAS_LAUNCH(k_chunk_totals, dim3(nchunks), dim3(SCAN_THREADS), st, (const uint32_t*)blk_cnt, nblk,
                 (const uint32_t*)nullptr, (const uint32_t*)nullptr, o.chunk_dups, (unsigned long long*)nullptr,
                 (uint32_t*)nullptr);
    // the kept count becomes the frame's duplicate count D
    TIGAS_LAUNCH(k_scan_dups, dim3(nchunks), dim3(SCAN_THREADS), st, (const uint32_t*)blk_cnt, nblk,
                 (const uint32_t*)o.chunk_dups, blk_off, nchunks, cnt);
    if (depth_out)
        TIGAS_LAUNCH((k_duplicate_culled<false, true>), dim3(nblk), dim3(K1_THREADS), st, sorted_rec, sorted_packed,
                     o.zkey, (const uint32_t*)blk_off, blk_cnt, (const uint32_t*)o.blk_view, (const Counters*)cnt,
                     views_dev, (const Rec*)o.rec, tile_w, tile_h, tile_out, val_out, depth_out);
    else
        TIGAS_LAUNCH((k_duplicate_culled<false, false>), dim3(nblk), dim3(K1_THREADS), st, sorted_rec, sorted_packed,
                     o.zkey, (const uint32_t*)blk_off, blk_cnt, (const uint32_t*)o.blk_view, (const Counters*)cnt,
                     views_dev, (const Rec*)o.rec, tile_w, tile_h, tile_out, val_out, depth_out);
}

int launch_sort(const SortBuffers& b, const SortPass* passes, int npasses, int which, uint32_t cap, int nblocks,
                int start, bool extra, Counters* cnt, const uint2* rect_src,
                uint2* rect_dst, hipStream_t st) {
    int cur = start;
    for (int p = 0; p < npasses; ++p) {
        const SortPass& ps = passes[p];
        const bool wide = ps.bits > 8;  // 9-bit digits: 512 per pass
        if (ps.adapt == 0)
            TIGAS_LAUNCH((k_sort_upsweep<512, true>), dim3(nblocks), dim3(SORT_THREADS), st,
                         (const uint32_t*)b.key[cur], cnt, which, cap, ps.shift, ps.bits, ps.adapt,
                         (const uint32_t*)b.zr, b.hist, nblocks, b.segmm);
        else if (wide)
            TIGAS_LAUNCH((k_sort_upsweep<512, false>), dim3(nblocks), dim3(SORT_THREADS), st,
                         (const uint32_t*)b.key[cur], cnt, which, cap, ps.shift, ps.bits, ps.adapt,
                         (const uint32_t*)b.zr, b.hist, nblocks, b.segmm);
        else
            TIGAS_LAUNCH((k_sort_upsweep<256, false>), dim3(nblocks), dim3(SORT_THREADS), st,
                         (const uint32_t*)b.key[cur], cnt, which, cap, ps.shift, ps.bits, ps.adapt,
                         (const uint32_t*)b.zr, b.hist, nblocks, b.segmm);
        const int ndig = 1 << ps.bits;
        // the first adaptive pass has one more workgroup: the key range
        const int nscan = ndig + (ps.adapt == 0 ? 1 : 0);
        if (nblocks <= 1024)
            TIGAS_LAUNCH(k_sort_scan<4>, dim3(nscan), dim3(256), st, b.hist, b.dtot, nblocks, ndig, ps.adapt, b.zr,
                         (const uint32_t*)b.segmm, cnt);
        else
            TIGAS_LAUNCH((k_sort_scan<SORT_MAX_BLOCKS / 256>), dim3(nscan), dim3(256), st, b.hist, b.dtot, nblocks,
                         ndig, ps.adapt, b.zr, (const uint32_t*)b.segmm, cnt);
        const bool sums = rect_src && p + 1 == npasses;
#define TIGAS_DOWN(E, S, N)                                                                                     \
    TIGAS_LAUNCH((k_sort_downsweep<E, S, N, N == 512 ? 512 : SORT_THREADS>), dim3(nblocks),                   \
                 dim3(N == 512 ? 512 : SORT_THREADS), st, b.key[cur], b.val[cur],                                 \
                 b.ext[cur], b.key[cur ^ 1], b.val[cur ^ 1], b.ext[cur ^ 1], cnt, which, cap, ps.shift, ps.bits, \
                 ps.adapt, (const uint32_t*)b.zr, (const uint32_t*)b.hist, (const uint32_t*)b.dtot, nblocks, rect_src, \
                 rect_dst)
        if (wide && extra && !sums) TIGAS_DOWN(true, false, 512);
        else if (wide) throw std::runtime_error("9-bit sort digits are for the packed-rectangle depth passes");
        else if (extra && sums) TIGAS_DOWN(true, true, 256);
        else if (extra) TIGAS_DOWN(true, false, 256);
        else if (sums) TIGAS_DOWN(false, true, 256);
        else TIGAS_DOWN(false, false, 256);
#undef TIGAS_DOWN
        cur ^= 1;
    }
    return cur;
}

void launch_tile_order(const uint2* ranges, uint32_t n_tiles, uint32_t* order, hipStream_t st) {
    if (n_tiles) TIGAS_LAUNCH(k_tile_order, dim3(1), dim3(256), st, ranges, n_tiles, order);
}

void launch_ranges(const uint32_t* tile_sorted, const Counters* cnt, uint32_t cap, uint2* ranges, Counters* host_cnt,
                   const PreOut& o, const ViewParams* views_dev, hipStream_t st) {
    // one 1024-word step per workgroup at capacity, but no more workgroups
    // than a large frame needs (the capacity may have been sized by a much
    // larger frame)
    TIGAS_LAUNCH(k_ranges, dim3(std::min<uint32_t>(16384u, std::max<uint32_t>(1u, (cap + 1023) / 1024))), dim3(256), st,
                 tile_sorted, cnt, cap, ranges, host_cnt);
}

uint32_t bin_emit_groups(uint32_t cap, uint32_t nrec) {
    const uint64_t max_cost = (uint64_t)cap + (uint64_t)BIN_ROUND_COST * ((nrec + 255) / 256);
    return std::max<uint32_t>(1u, (uint32_t)((max_cost + BIN_PAIRS - 1) / BIN_PAIRS));
}

bool bin_fits(int tiles_x, int tiles_y) {
    return tiles_x >= 1 && tiles_y >= 1 && tiles_x <= 255 && tiles_y <= 255 &&
           (tiles_x + 1) * (tiles_y + 1) <= BIN_GRID_MAX && tiles_x * tiles_y <= BIN_TILES_MAX;
}

void launch_bin(const uint32_t* sorted_rec, const uint32_t* sorted_packed, const Counters* cnt, uint32_t nrec,
                uint32_t cap, int tiles_x, int tiles_y, uint32_t* hist, uint32_t* gsum, uint32_t* round_cnt,
                uint32_t* round_off, uint2* ranges, Counters* host_cnt, const PreOut& o, const ViewParams* views_dev,
                uint32_t* val_out, uint32_t* tile_out, uint32_t* depth_out, uint32_t* order, hipStream_t st) {
    const uint32_t n_tiles = (uint32_t)(tiles_x * tiles_y);
    const uint32_t nbc = std::max<uint32_t>(1u, (nrec + BIN_BLOCK - 1) / BIN_BLOCK);
    // after the BIN_GROUPS + 2 rows of gsum: the 256-tile chunk totals, the
    // histogram blocks' entry totals, then the first-round table
    uint32_t* tchunk = gsum + (size_t)(BIN_GROUPS + 2) * n_tiles;
    uint32_t* blk_tot = tchunk + BIN_TILES_MAX / 256;
    uint32_t* start_round = blk_tot + nbc;
    TIGAS_LAUNCH(k_bin_hist, dim3(nbc), dim3(256), st, sorted_packed, cnt, tiles_x, tiles_y, hist, round_cnt, blk_tot);
    TIGAS_LAUNCH(k_bin_prefix, dim3((n_tiles + 255) / 256, BIN_GROUPS), dim3(256), st, hist, cnt, n_tiles, gsum);
    TIGAS_LAUNCH(k_bin_groups, dim3((n_tiles + 255) / 256), dim3(256), st, gsum, cnt, n_tiles, tchunk);
    // enough emission workgroups for the largest cost the capacities allow
    const uint32_t nwg = bin_emit_groups(cap, nrec);
    const uint32_t ntc = (n_tiles + 255) / 256, nrc = std::max<uint32_t>(1u, (nrec + 255) / 256 / 256 + 1);
    TIGAS_LAUNCH(k_bin_tiles, dim3(ntc + nrc), dim3(256), st, gsum, cnt, n_tiles, ranges, (const uint32_t*)round_cnt,
                 round_off, start_round, nwg, host_cnt, (const uint32_t*)tchunk, (const uint32_t*)blk_tot);
    const size_t ncell = (size_t)(tiles_x + 1) * (tiles_y + 1);
    const size_t lds = 8 * 4 * (size_t)(tiles_x + 1 + tiles_y + 1) + 4 * ncell;
    // one more workgroup: the blend's dispatch order
    if (tile_out)
        TIGAS_LAUNCH_SHM(k_bin_emit<true>, dim3(nwg + 1), dim3(256), lds, st, (const uint2*)ranges, order, sorted_rec,
                         sorted_packed, cnt,
                         (const uint32_t*)hist, (const uint32_t*)gsum, (const uint32_t*)round_off,
                         (const uint32_t*)start_round, tiles_x, tiles_y, val_out, tile_out, depth_out,
                         (const uint32_t*)o.zkey);
    else
        TIGAS_LAUNCH_SHM(k_bin_emit<false>, dim3(nwg + 1), dim3(256), lds, st, (const uint2*)ranges, order,
                         sorted_rec, sorted_packed, cnt,
                         (const uint32_t*)hist, (const uint32_t*)gsum, (const uint32_t*)round_off,
                         (const uint32_t*)start_round, tiles_x, tiles_y, val_out, tile_out, depth_out,
                         (const uint32_t*)o.zkey);
}

template <int TW, int TH, int BD, int PPL>
static void blend_launch(const BlendArgs& A, bool count, uint32_t* queue, int persistent_blocks, hipStream_t st) {
    if (queue) {
        TIGAS_LAUNCH((k_blend_persistent<TW, TH, BD, PPL>), dim3(persistent_blocks), dim3(TW * TH / PPL), st, A,
                     queue);
    } else {
        const uint32_t per_round = 8 * BLEND_CHUNK;  // one chunk for every XCD
        const uint32_t tiles = ((A.n_tiles + per_round - 1) / per_round) * per_round;
        const dim3 grid(tiles);
        if (count) TIGAS_LAUNCH((k_blend<TW, TH, BD, PPL, true>), grid, dim3(TW * TH / PPL), st, A);
        else TIGAS_LAUNCH((k_blend<TW, TH, BD, PPL, false>), grid, dim3(TW * TH / PPL), st, A);
    }
}

template <int TW, int TH, int PPL>
static void blend_bd(int bd, const BlendArgs& A, bool count, uint32_t* queue, int pb, hipStream_t st) {
    switch (bd) {
        case 128: blend_launch<TW, TH, 2, PPL>(A, count, queue, pb, st); break;
        case 256: blend_launch<TW, TH, 4, PPL>(A, count, queue, pb, st); break;
        default: blend_launch<TW, TH, 1, PPL>(A, count, queue, pb, st); break;
    }
}

void launch_blend(const ViewParams* views_dev, int nviews, uint32_t n_tiles, const uint2* ranges,
                  const uint32_t* vals, const PreOut& o, uint32_t nrec, int tile_w, int tile_h, int batch_depth,
                  int ppl, unsigned long long* work, uint32_t* queue, int persistent_blocks, bool cull,
                  const uint32_t* order, hipStream_t st) {
    if (n_tiles == 0) return;
    const BlendArgs A{views_dev, nviews, n_tiles, ranges, vals, o.rec, nrec, work, cull ? 1 : 0, order};
    const bool count = work != nullptr;
    if (count) queue = nullptr;
    const bool two = ppl == 2 && tile_h >= 16;
    if (tile_w == 8 && tile_h == 8) blend_bd<8, 8, 1>(batch_depth, A, count, queue, persistent_blocks, st);
    else if (tile_w == 16 && tile_h == 32) {
        if (two) blend_bd<16, 32, 2>(batch_depth, A, count, queue, persistent_blocks, st);
        else blend_bd<16, 32, 1>(batch_depth, A, count, queue, persistent_blocks, st);
    } else if (tile_w == 32 && tile_h == 16) {
        if (two) blend_bd<32, 16, 2>(batch_depth, A, count, queue, persistent_blocks, st);
        else blend_bd<32, 16, 1>(batch_depth, A, count, queue, persistent_blocks, st);
    } else {
        if (two) blend_bd<16, 16, 2>(batch_depth, A, count, queue, persistent_blocks, st);
        else blend_bd<16, 16, 1>(batch_depth, A, count, queue, persistent_blocks, st);
    }
}

// Resident workgroups per CU of the persistent blend kernel for a configuration.
int blend_persistent_occupancy(int tile_w, int tile_h, int batch_depth, int ppl) {
    int n = 0;
    const int bd = batch_depth == 128 ? 2 : (batch_depth == 256 ? 4 : 1);
    const bool two = ppl == 2 && tile_h >= 16;
#define TIGAS_OCC3(TW, TH, P)                                                                                       \
    do {                                                                                                           \
        if (bd == 1) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_persistent<TW, TH, 1, P>,       \
                                                                         TW * TH / P, 0);                          \
        else if (bd == 2) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_persistent<TW, TH, 2, P>,  \
                                                                              TW * TH / P, 0);                     \
        else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_persistent<TW, TH, 4, P>, TW * TH / P,  \
                                                                 0);                                               \
    } while (0)
    if (tile_w == 8 && tile_h == 8) TIGAS_OCC3(8, 8, 1);
    else if (tile_w == 16 && tile_h == 32) { if (two) TIGAS_OCC3(16, 32, 2); else TIGAS_OCC3(16, 32, 1); }
    else if (tile_w == 32 && tile_h == 16) { if (two) TIGAS_OCC3(32, 16, 2); else TIGAS_OCC3(32, 16, 1); }
    else { if (two) TIGAS_OCC3(16, 16, 2); else TIGAS_OCC3(16, 16, 1); }
#undef TIGAS_OCC3
    return n > 0 ? n : 1;
}

void launch_wave_scan_selftest(const uint32_t* in, uint32_t* out, int n, hipStream_t st) {
    TIGAS_LAUNCH(k_wave_scan_selftest, dim3((n + 63) / 64), dim3(64), st, in, out, n);
}

}  // namespace tigas

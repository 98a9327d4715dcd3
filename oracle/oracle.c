/*
 * FP64 CPU oracle of the forward 3D Gaussian Splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path loads this file:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code with the HIP library.
 *
 * What it computes is the plain definition of the rendered frame, with no
 * tiling, no sorting structure beyond one global depth order and no blocking:
 *
 *   per Gaussian (Section 5.1, "PLY Model and Primitives"):
 *     scale = exp(log-scale), opacity = sigmoid(logit), rotation from the
 *     normalised quaternion (w,x,y,z), 3D covariance R S S^T R^T;
 *     view-dependent colour from real spherical harmonics up to degree 3,
 *     evaluated at the unit direction from the camera centre to the Gaussian,
 *     plus 0.5 and clamped below at 0.
 *   camera (Section 5.1, "Rendering Engine"):
 *     T_w->c = [R^T, -R^T t]; p_c = R^T (mu - t);
 *     lambda [u v 1]^T = K p_c with lambda = z_c.
 *   EWA splatting of the 3D covariance to the image plane (the representation
 *   of Kerbl et al. 2023 that the paper builds on):  J V Sigma V^T J^T with the
 *   perspective Jacobian J, plus a 0.3 px^2 low-pass term on the diagonal;
 *   conic = inverse of the 2D covariance.
 *   per pixel, Gaussians in ascending depth order, starting from T = 1, C = 0:
 *     alpha = min(0.99, o * exp(-0.5 d^T conic d)), d = pixel centre - (u,v);
 *     alpha < 1/255: skipped;  T' = T (1 - alpha) < 1e-4: stop, this Gaussian
 *     excluded;  otherwise C += alpha T rgb, T = T';  pixel = C + T bg.
 *   8-bit frame (Section 5.1, final rasterized frames): each channel
 *     round-half-up(255 * clamp(c, 0, 1)), in FP32.
 *
 * Readings taken where the paper is silent (each one is listed with its reason
 * in the design notes of the repository):
 *   - pixel (i, j) is sampled at its centre (i + 0.5, j + 0.5);
 *   - R is camera-to-world, camera axes x right, y down, z forward;
 *   - the depth order key is the FP32 value
 *       z32 = fmaf(V20, mx, fmaf(V21, my, fmaf(V22, mz, tz)))
 *     with V = R^T and tz = float((-R^T t)_z) rounded once from FP64; ties are
 *     broken by Gaussian index; z32 is used only to order and to cull at the
 *     near plane (z32 <= 0.2 dropped); every other value is FP64;
 *   - the Jacobian uses x/z and y/z clamped to 1.3x the half field of view;
 *   - the thresholds 0.99, 1/255 and 1e-4 are the FP32 constants promoted
 *     exactly to FP64, compared strictly as stated;
 *   - a Gaussian with a non-finite attribute or a zero quaternion is dropped.
 *
 * Set-valued result.  The GPU computes in FP32; where a threshold decision of
 * the FP64 oracle has a margin inside a small band (|alpha - 1/255| or
 * |T' - 1e-4|, relative band widths given by the caller), the oracle follows
 * both outcomes and reports every branch's (C, T).  A pixel is correct if it
 * matches any branch.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NF 16
enum { F_U, F_V, F_Z, F_A, F_B, F_C, F_CA, F_CB, F_CC, F_OP, F_R, F_G, F_BL, F_EX, F_EY, F_DET };

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- camera -- */

/* Output size and intrinsics for a resolution-scaled render (the paper's ABR
 * ladder renders downscaled frames and re-centres the principal point).
 * out = round-half-up(size * s); the intrinsics are multiplied by the ratio of
 * output to full size and rounded to FP32, the precision of the interface. */
void orc_rung(double fx, double fy, double cx, double cy, int width, int height, double s,
              int* out_w, int* out_h, double* k4) {
    int w = (int)floor(width * s + 0.5);
    int h = (int)floor(height * s + 0.5);
    double rx = (double)w / (double)width, ry = (double)h / (double)height;
    *out_w = w;
    *out_h = h;
    k4[0] = (double)(float)(fx * rx);
    k4[1] = (double)(float)(fy * ry);
    k4[2] = (double)(float)(cx * rx);
    k4[3] = (double)(float)(cy * ry);
}

/* ------------------------------------------------------ spherical harmonics */

/* Real spherical harmonics with the Condon-Shortley phase, l = 0..3,
 * m = -l..l, evaluated at a unit vector (x, y, z), using the textbook
 * Cartesian polynomials and normalisations. */
void orc_sh_basis(const double d[3], double Y[16]) {
    double x = d[0], y = d[1], z = d[2];
    double c0 = 0.5 * sqrt(1.0 / PI);
    double c1 = sqrt(3.0 / (4.0 * PI));
    double c2a = 0.5 * sqrt(15.0 / PI), c2b = 0.25 * sqrt(5.0 / PI), c2c = 0.25 * sqrt(15.0 / PI);
    double c3a = 0.25 * sqrt(35.0 / (2.0 * PI)), c3b = 0.5 * sqrt(105.0 / PI);
    double c3c = 0.25 * sqrt(21.0 / (2.0 * PI)), c3d = 0.25 * sqrt(7.0 / PI), c3e = 0.25 * sqrt(105.0 / PI);
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (3.0 * z * z - 1.0);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    Y[9] = -c3a * y * (3.0 * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (5.0 * z * z - 1.0);
    Y[12] = c3d * z * (5.0 * z * z - 3.0);
    Y[13] = -c3c * x * (5.0 * z * z - 1.0);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.0 * y * y);
}

void orc_sh_basis_many(int64_t n, const double* dirs, double* Y) {
    for (int64_t i = 0; i < n; ++i) orc_sh_basis(dirs + 3 * i, Y + 16 * i);
}

/* colour = max(0, 0.5 + sum_{i < (deg+1)^2} Y_i k_i) per channel;
 * k is [16][3] coefficient-major. */
void orc_sh_color(int deg, const double d[3], const double* k, double rgb[3]) {
    double Y[16];
    orc_sh_basis(d, Y);
    int nc = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double s = 0.5;
        for (int i = 0; i < nc; ++i) s += Y[i] * k[i * 3 + ch];
        rgb[ch] = s > 0.0 ? s : 0.0;
    }
}

/* ------------------------------------------------------------ preprocess -- */

static int all_finite(const float* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

/* Per-Gaussian FP64 projection.  cam = {fx, fy, cx, cy, W, H} of the output
 * image (already rung-scaled).  Writes ORC_NF doubles per Gaussian, the FP32
 * order-key bits and a validity flag.  Returns the number of valid Gaussians. */
int64_t orc_preprocess(int64_t n, const float* means, const float* log_scales, const float* quats,
                       const float* opacity_logits, const float* sh, int sh_degree,
                       const float* Rcw, const float* tcam, const double* cam,
                       double* out, uint32_t* zkey, uint8_t* valid) {
    double fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3], W = cam[4], H = cam[5];
    double V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = (double)Rcw[j * 3 + i]; /* V = R^T */
    double t[3] = {tcam[0], tcam[1], tcam[2]};
    double twc_z = -(V[2][0] * t[0] + V[2][1] * t[1] + V[2][2] * t[2]);
    float tz32 = (float)twc_z;
    float v20 = (float)V[2][0], v21 = (float)V[2][1], v22 = (float)V[2][2];
    double lim_x = 1.3 * fmax(cx, W - cx) / fx;
    double lim_y = 1.3 * fmax(cy, H - cy) / fy;
    int64_t nvalid = 0;

#pragma omp parallel for schedule(static, 4096) reduction(+ : nvalid)
    for (int64_t g = 0; g < n; ++g) {
        double* o = out + g * ORC_NF;
        for (int f = 0; f < ORC_NF; ++f) o[f] = 0.0;
        const float* mu32 = means + 3 * g;
        const float* q32 = quats + 4 * g;
        const float* ls32 = log_scales + 3 * g;
        int ok = all_finite(mu32, 3) && all_finite(q32, 4) && all_finite(ls32, 3) &&
                 isfinite(opacity_logits[g]) && all_finite(sh + 48 * g, 3 * (sh_degree + 1) * (sh_degree + 1));

        float z32 = fmaf(v20, mu32[0], fmaf(v21, mu32[1], fmaf(v22, mu32[2], tz32)));
        uint32_t zb;
        memcpy(&zb, &z32, 4);
        zkey[g] = zb;
        if (!(z32 > 0.2f)) ok = 0;

        double qw = q32[0], qx = q32[1], qy = q32[2], qz = q32[3];
        double qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
        if (!(qn2 > 0.0)) ok = 0;
        if (!ok) {
            valid[g] = 0;
            continue;
        }

        /* camera-space centre */
        double d[3] = {mu32[0] - t[0], mu32[1] - t[1], mu32[2] - t[2]};
        double pc[3];
        for (int i = 0; i < 3; ++i) pc[i] = V[i][0] * d[0] + V[i][1] * d[1] + V[i][2] * d[2];
        double x = pc[0], y = pc[1], z = pc[2];

        /* 3D covariance Sigma = Rq S S^T Rq^T */
        double inv = 1.0 / sqrt(qn2);
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
        double Rq[3][3] = {
            {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
            {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
            {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
        double s[3] = {exp((double)ls32[0]), exp((double)ls32[1]), exp((double)ls32[2])};
        double M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = Rq[i][j] * s[j];
        double Sig[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Sig[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];

        /* perspective Jacobian at the (clamped) centre direction */
        double rx = x / z, ry = y / z;
        rx = fmin(fmax(rx, -lim_x), lim_x);
        ry = fmin(fmax(ry, -lim_y), lim_y);
        double J[2][3] = {{fx / z, 0.0, -fx * rx / z}, {0.0, fy / z, -fy * ry / z}};
        double T[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) T[i][j] = J[i][0] * V[0][j] + J[i][1] * V[1][j] + J[i][2] * V[2][j];
        double TS[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) TS[i][j] = T[i][0] * Sig[0][j] + T[i][1] * Sig[1][j] + T[i][2] * Sig[2][j];
        double a = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + 0.3;
        double b = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
        double c = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + 0.3;
        double det = a * c - b * b;
        if (!(det > 0.0) || !isfinite(det)) {
            valid[g] = 0;
            continue;
        }

        double op = 1.0 / (1.0 + exp(-(double)opacity_logits[g]));

        /* colour: SH at the unit direction camera centre -> Gaussian (world) */
        double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double dir[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
        double k[48];
        for (int i = 0; i < 48; ++i) k[i] = (double)sh[48 * g + i];
        double rgb[3];
        orc_sh_color(sh_degree, dir, k, rgb);

        /* support of alpha >= 1/255: Q <= 2 ln(255 o); its bounding box */
        double k2 = 2.0 * log(255.0 * op);
        double ex = k2 > 0.0 ? sqrt(k2 * a) : 0.0;
        double ey = k2 > 0.0 ? sqrt(k2 * c) : 0.0;

        o[F_U] = fx * x / z + cx;
        o[F_V] = fy * y / z + cy;
        o[F_Z] = z;
        o[F_A] = a;
        o[F_B] = b;
        o[F_C] = c;
        o[F_CA] = c / det;
        o[F_CB] = -b / det;
        o[F_CC] = a / det;
        o[F_OP] = op;
        o[F_R] = rgb[0];
        o[F_G] = rgb[1];
        o[F_BL] = rgb[2];
        o[F_EX] = ex;
        o[F_EY] = ey;
        o[F_DET] = det;
        valid[g] = 1;
        ++nvalid;
    }
    return nvalid;
}

/* -------------------------------------------------------------- ordering -- */

static int cmp_u64(const void* pa, const void* pb) {
    uint64_t a = *(const uint64_t*)pa, b = *(const uint64_t*)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Indices of valid Gaussians in ascending (z32 key, index) order.  All valid
 * keys are positive FP32 values, whose bit patterns order like the values. */
int64_t orc_depth_order(int64_t n, const uint32_t* zkey, const uint8_t* valid, int64_t* order) {
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t g = 0; g < n; ++g)
        if (valid[g]) tmp[m++] = ((uint64_t)zkey[g] << 32) | (uint64_t)(uint32_t)g;
    qsort(tmp, (size_t)m, sizeof(uint64_t), cmp_u64);
    for (int64_t i = 0; i < m; ++i) order[i] = (int64_t)(tmp[i] & 0xffffffffu);
    free(tmp);
    return m;
}

/* ---------------------------------------------------------------- blend -- */

typedef struct {
    int64_t nv;
    const double* pre; /* nv x ORC_NF in depth order */
    const double* box; /* nv x 4 prefilter box (xlo, xhi, ylo, yhi), or NULL */
    double px, py;
    double bg[3];
    double band_a, band_t;
    int maxb, nb, unresolved;
    double* out; /* maxb x 4 : r, g, b, T */
} blend_ctx;

static const double A_MAX = (double)0.99f;
static const double A_MIN = (double)(1.0f / 255.0f);
static const double T_MIN = (double)1e-4f;

static void emit(blend_ctx* cx, const double C[3], double T) {
    if (cx->nb >= cx->maxb) {
        cx->unresolved = 1;
        return;
    }
    double* o = cx->out + 4 * cx->nb;
    o[0] = C[0] + T * cx->bg[0];
    o[1] = C[1] + T * cx->bg[1];
    o[2] = C[2] + T * cx->bg[2];
    o[3] = T;
    cx->nb++;
}

/* reserve room for one more branch; 0 if the branch budget is spent */
static int can_fork(blend_ctx* cx, int pending) {
    if (cx->nb + pending + 1 >= cx->maxb) {
        cx->unresolved = 1;
        return 0;
    }
    return 1;
}

static void blend_from(blend_ctx* cx, int64_t k, double T, const double Cin[3], int pending) {
    double C[3] = {Cin[0], Cin[1], Cin[2]};
    for (; k < cx->nv; ++k) {
        if (cx->box) {
            const double* bx = cx->box + 4 * k;
            if (cx->px < bx[0] || cx->px > bx[1] || cx->py < bx[2] || cx->py > bx[3]) continue;
        }
        const double* g = cx->pre + k * ORC_NF;
        double dx = cx->px - g[F_U], dy = cx->py - g[F_V];
        double Q = g[F_CA] * dx * dx + 2.0 * g[F_CB] * dx * dy + g[F_CC] * dy * dy;
        double alpha = g[F_OP] * exp(-0.5 * Q);
        if (alpha > A_MAX) alpha = A_MAX;

        if (fabs(alpha - A_MIN) <= cx->band_a * A_MIN && can_fork(cx, pending)) {
            /* near the skip threshold: follow "skipped" here, "taken" below */
            blend_from(cx, k + 1, T, C, pending + 1);
        } else if (alpha < A_MIN) {
            continue;
        }
        double Tn = T * (1.0 - alpha);
        if (fabs(Tn - T_MIN) <= cx->band_t * T_MIN && can_fork(cx, pending)) {
            /* near the stop threshold: record "stopped", continue as "not stopped" */
            emit(cx, C, T);
        } else if (Tn < T_MIN) {
            emit(cx, C, T);
            return;
        }
        double w = alpha * T;
        C[0] += w * g[F_R];
        C[1] += w * g[F_G];
        C[2] += w * g[F_BL];
        T = Tn;
    }
    emit(cx, C, T);
}

/* Build the conservative prefilter box of each Gaussian in depth order: a
 * pixel centre outside it has Q > 2 ln(o / alpha_lo) with alpha_lo below the
 * skip band, i.e. the Gaussian is skipped there with certainty (Q >= dx^2/a and
 * Q >= dy^2/c for any offset). */
void orc_prefilter_boxes(int64_t nv, const double* pre, double band_a, double* box) {
    double a_lo = A_MIN * (1.0 - 2.0 * band_a);
    for (int64_t k = 0; k < nv; ++k) {
        const double* g = pre + k * ORC_NF;
        double k2 = 2.0 * log(g[F_OP] / a_lo);
        double* b = box + 4 * k;
        if (!(k2 > 0.0)) {
            b[0] = 1.0;
            b[1] = -1.0;
            b[2] = 1.0;
            b[3] = -1.0;
            continue;
        }
        double ex = sqrt(k2 * g[F_A]) * (1.0 + 1e-9) + 1e-9;
        double ey = sqrt(k2 * g[F_C]) * (1.0 + 1e-9) + 1e-9;
        b[0] = g[F_U] - ex;
        b[1] = g[F_U] + ex;
        b[2] = g[F_V] - ey;
        b[3] = g[F_V] + ey;
    }
}

/* Render the pixels (px[i], py[i]) (integer pixel indices, sampled at their
 * centres).  pre: nv x ORC_NF per-Gaussian values in depth order.  box: the
 * prefilter boxes or NULL for plain brute force.  out: npix x maxb x 4,
 * nbranch: number of branches per pixel, negated when the branch budget was
 * exceeded (unresolved). */
void orc_render_pixels(int64_t nv, const double* pre, const double* box, int64_t npix, const int32_t* px,
                       const int32_t* py, const double* bg, double band_a, double band_t, int maxb,
                       double* out, int32_t* nbranch) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < npix; ++i) {
        blend_ctx cx;
        cx.nv = nv;
        cx.pre = pre;
        cx.box = box;
        cx.px = (double)px[i] + 0.5;
        cx.py = (double)py[i] + 0.5;
        cx.bg[0] = bg[0];
        cx.bg[1] = bg[1];
        cx.bg[2] = bg[2];
        cx.band_a = band_a;
        cx.band_t = band_t;
        cx.maxb = maxb;
        cx.nb = 0;
        cx.unresolved = 0;
        cx.out = out + (size_t)i * (size_t)maxb * 4;
        double C0[3] = {0.0, 0.0, 0.0};
        blend_from(&cx, 0, 1.0, C0, 0);
        nbranch[i] = cx.unresolved ? -cx.nb : cx.nb;
    }
}

/* ------------------------------------------------------------ 8-bit frame -- */

/* The frame leaves the renderer as 8 bits per channel (Section 5.1, final
 * rasterized frames).  Reading: each FP32 channel value c maps to
 * floor(min(max(c, 0), 1) * 255 + 0.5), evaluated in FP32 (one rounded
 * product, one rounded sum), i.e. round half up on [0, 255]. */
void orc_pack_rgb8(int64_t n, const float* in, uint8_t* out) {
    for (int64_t i = 0; i < n; ++i) {
        float c = in[i];
        if (!(c > 0.0f)) c = 0.0f; /* also maps NaN to 0 */
        if (c > 1.0f) c = 1.0f;
        volatile float scaled = c * 255.0f;
        volatile float shifted = scaled + 0.5f;
        out[i] = (uint8_t)floorf(shifted);
    }
}

/* Number of OpenMP threads the pixel loops use from now on (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

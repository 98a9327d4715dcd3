/* JPEG oracle: test infrastructure only (the tests and the benchmark's
 * CPU-baseline leg use it; nothing in the product links it).
 *
 * A baseline sequential JPEG (ITU-T T.81 with a JFIF header) of an RGB8
 * frame, the per-frame payload that the paper's backend returns for a
 * request at a quality level of its bitrate ladder (Table 1: 10, 35, 65 and
 * 90).  Written step by step from the standard; where the standard leaves a
 * choice this file fixes it, and the GPU encoder makes the same choices, so
 * its bytes must equal these:
 *   - colour: full-range YCbCr (JFIF), computed in FP32 as written below,
 *     level shift by 128 (for Cb and Cr the +128 offset and the shift cancel);
 *   - sampling 4:4:4, one 8x8 block per component per MCU, the last column
 *     and row of pixels repeated to fill whole blocks;
 *   - forward DCT: orthonormal 8x8 DCT-II, F = M f M^T with
 *     M[k][n] = c(k)/2 cos((2n+1)k pi/16) (c(0) = 1/sqrt 2, else 1) rounded
 *     once from FP64 to FP32; every sum is an FMA chain in index order
 *     starting from zero, over the columns first, then over the rows;
 *   - quantisation: x = F * (1/Q) in FP32, q = trunc(x + copysign(1/2, x)),
 *     AC values clamped to +-1023 (baseline range);
 *   - tables: the luminance and chrominance quantisation tables of Annex K
 *     scaled by quality the usual way (s = 5000/q below 50, else 200 - 2q;
 *     entry (base s + 50) / 100 clamped to 1..255) and the four Huffman
 *     tables of Annex K;
 *   - entropy coding of Annex F (DC difference category + magnitude bits;
 *     AC run/size symbols with ZRL and EOB), 0xFF bytes followed by 0x00,
 *     pad bits set to 1;
 *   - restart intervals of 40 MCUs in raster order (DRI), RSTn after every
 *     interval but the last, DC predictions reset to zero at each interval.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RESTART_MCUS 40

/* Annex K, Table K.1 and K.2, rows of the 8x8 block (natural order) */
static const uint8_t QL[64] = {16, 11, 10, 16, 24,  40,  51,  61,  12, 12, 14, 19, 26,  58,  60,  55,
                               14, 13, 16, 24, 40,  57,  69,  56,  14, 17, 22, 29, 51,  87,  80,  62,
                               18, 22, 37, 56, 68,  109, 103, 77,  24, 35, 55, 64, 81,  104, 113, 92,
                               49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99};
static const uint8_t QC[64] = {17, 18, 24, 47, 99, 99, 99, 99, 18, 21, 26, 66, 99, 99, 99, 99,
                               24, 26, 56, 99, 99, 99, 99, 99, 47, 66, 99, 99, 99, 99, 99, 99,
                               99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99,
                               99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99};

/* Annex K, Tables K.3 to K.6: code counts per length 1..16, then the symbols */
static const uint8_t DCL_N[16] = {0, 1, 5, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0};
static const uint8_t DCC_N[16] = {0, 3, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0};
static const uint8_t DC_SYM[12] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
static const uint8_t ACL_N[16] = {0, 2, 1, 3, 3, 2, 4, 3, 5, 5, 4, 4, 0, 0, 1, 0x7d};
static const uint8_t ACL_SYM[162] = {
    0x01, 0x02, 0x03, 0x00, 0x04, 0x11, 0x05, 0x12, 0x21, 0x31, 0x41, 0x06, 0x13, 0x51, 0x61, 0x07, 0x22, 0x71,
    0x14, 0x32, 0x81, 0x91, 0xa1, 0x08, 0x23, 0x42, 0xb1, 0xc1, 0x15, 0x52, 0xd1, 0xf0, 0x24, 0x33, 0x62, 0x72,
    0x82, 0x09, 0x0a, 0x16, 0x17, 0x18, 0x19, 0x1a, 0x25, 0x26, 0x27, 0x28, 0x29, 0x2a, 0x34, 0x35, 0x36, 0x37,
    0x38, 0x39, 0x3a, 0x43, 0x44, 0x45, 0x46, 0x47, 0x48, 0x49, 0x4a, 0x53, 0x54, 0x55, 0x56, 0x57, 0x58, 0x59,
    0x5a, 0x63, 0x64, 0x65, 0x66, 0x67, 0x68, 0x69, 0x6a, 0x73, 0x74, 0x75, 0x76, 0x77, 0x78, 0x79, 0x7a, 0x83,
    0x84, 0x85, 0x86, 0x87, 0x88, 0x89, 0x8a, 0x92, 0x93, 0x94, 0x95, 0x96, 0x97, 0x98, 0x99, 0x9a, 0xa2, 0xa3,
    0xa4, 0xa5, 0xa6, 0xa7, 0xa8, 0xa9, 0xaa, 0xb2, 0xb3, 0xb4, 0xb5, 0xb6, 0xb7, 0xb8, 0xb9, 0xba, 0xc2, 0xc3,
    0xc4, 0xc5, 0xc6, 0xc7, 0xc8, 0xc9, 0xca, 0xd2, 0xd3, 0xd4, 0xd5, 0xd6, 0xd7, 0xd8, 0xd9, 0xda, 0xe1, 0xe2,
    0xe3, 0xe4, 0xe5, 0xe6, 0xe7, 0xe8, 0xe9, 0xea, 0xf1, 0xf2, 0xf3, 0xf4, 0xf5, 0xf6, 0xf7, 0xf8, 0xf9, 0xfa};
static const uint8_t ACC_N[16] = {0, 2, 1, 2, 4, 4, 3, 4, 7, 5, 4, 4, 0, 1, 2, 0x77};
static const uint8_t ACC_SYM[162] = {
    0x00, 0x01, 0x02, 0x03, 0x11, 0x04, 0x05, 0x21, 0x31, 0x06, 0x12, 0x41, 0x51, 0x07, 0x61, 0x71, 0x13, 0x22,
    0x32, 0x81, 0x08, 0x14, 0x42, 0x91, 0xa1, 0xb1, 0xc1, 0x09, 0x23, 0x33, 0x52, 0xf0, 0x15, 0x62, 0x72, 0xd1,
    0x0a, 0x16, 0x24, 0x34, 0xe1, 0x25, 0xf1, 0x17, 0x18, 0x19, 0x1a, 0x26, 0x27, 0x28, 0x29, 0x2a, 0x35, 0x36,
    0x37, 0x38, 0x39, 0x3a, 0x43, 0x44, 0x45, 0x46, 0x47, 0x48, 0x49, 0x4a, 0x53, 0x54, 0x55, 0x56, 0x57, 0x58,
    0x59, 0x5a, 0x63, 0x64, 0x65, 0x66, 0x67, 0x68, 0x69, 0x6a, 0x73, 0x74, 0x75, 0x76, 0x77, 0x78, 0x79, 0x7a,
    0x82, 0x83, 0x84, 0x85, 0x86, 0x87, 0x88, 0x89, 0x8a, 0x92, 0x93, 0x94, 0x95, 0x96, 0x97, 0x98, 0x99, 0x9a,
    0xa2, 0xa3, 0xa4, 0xa5, 0xa6, 0xa7, 0xa8, 0xa9, 0xaa, 0xb2, 0xb3, 0xb4, 0xb5, 0xb6, 0xb7, 0xb8, 0xb9, 0xba,
    0xc2, 0xc3, 0xc4, 0xc5, 0xc6, 0xc7, 0xc8, 0xc9, 0xca, 0xd2, 0xd3, 0xd4, 0xd5, 0xd6, 0xd7, 0xd8, 0xd9, 0xda,
    0xe2, 0xe3, 0xe4, 0xe5, 0xe6, 0xe7, 0xe8, 0xe9, 0xea, 0xf2, 0xf3, 0xf4, 0xf5, 0xf6, 0xf7, 0xf8, 0xf9, 0xfa};

/* zig-zag scan (Figure A.6): scan position -> row-major index, by walking
   the anti-diagonals, upwards on even ones and downwards on odd ones */
static void zigzag(int zz[64]) {
    int i = 0;
    for (int d = 0; d < 15; ++d) {
        const int hi = d < 8 ? d : 7, lo = d < 8 ? 0 : d - 7;
        for (int j = hi; j >= lo; --j) {
            const int row = (d % 2 == 0) ? j : d - j;
            zz[i++] = row * 8 + (d - row);
        }
    }
}

void orc_jpeg_qtable(int quality, int chroma, uint8_t out[64]) {
    const int q = quality < 1 ? 1 : (quality > 100 ? 100 : quality);
    const long s = q < 50 ? 5000 / q : 200 - 2 * q;
    const uint8_t* base = chroma ? QC : QL;
    for (int i = 0; i < 64; ++i) {
        long v = ((long)base[i] * s + 50) / 100;
        out[i] = (uint8_t)(v < 1 ? 1 : (v > 255 ? 255 : v));
    }
}

/* code counts and symbols of table t: 0 DC luma, 1 AC luma, 2 DC chroma, 3 AC chroma */
int orc_jpeg_htable(int t, uint8_t counts[16], uint8_t syms[162]) {
    const uint8_t* n = t == 0 ? DCL_N : t == 1 ? ACL_N : t == 2 ? DCC_N : ACC_N;
    const uint8_t* v = (t & 1) ? (t == 1 ? ACL_SYM : ACC_SYM) : DC_SYM;
    int total = 0;
    for (int i = 0; i < 16; ++i) total += n[i];
    memcpy(counts, n, 16);
    memcpy(syms, v, (size_t)total);
    return total;
}

/* canonical codes (Annex C): consecutive codes within a length, doubled
   between lengths */
typedef struct {
    uint16_t code[256];
    uint8_t len[256];
} huff_t;
static void huff_build(const uint8_t n[16], const uint8_t* sym, huff_t* h) {
    memset(h, 0, sizeof *h);
    unsigned code = 0;
    int k = 0;
    for (int l = 1; l <= 16; ++l) {
        for (int i = 0; i < n[l - 1]; ++i, ++k) {
            h->code[sym[k]] = (uint16_t)code++;
            h->len[sym[k]] = (uint8_t)l;
        }
        code <<= 1;
    }
}

typedef struct {
    uint8_t* buf;
    int64_t cap, n;
    unsigned acc;
    int nacc;
} bw_t;
static void put_byte(bw_t* w, uint8_t b) {
    if (w->n < w->cap) w->buf[w->n] = b;
    w->n++;
}
static void put_bits(bw_t* w, unsigned v, int nb) { /* most significant bit first */
    for (int i = nb - 1; i >= 0; --i) {
        w->acc = (w->acc << 1) | ((v >> i) & 1u);
        if (++w->nacc == 8) {
            const uint8_t b = (uint8_t)w->acc;
            put_byte(w, b);
            if (b == 0xFF) put_byte(w, 0x00);
            w->acc = 0;
            w->nacc = 0;
        }
    }
}
static void pad_ones(bw_t* w) {
    while (w->nacc) put_bits(w, 1u, 1);
}
static void put16(bw_t* w, unsigned v) {
    put_byte(w, (uint8_t)(v >> 8));
    put_byte(w, (uint8_t)v);
}
static int magnitude_bits(int v) {
    unsigned a = (unsigned)(v < 0 ? -v : v);
    int n = 0;
    while (a) {
        ++n;
        a >>= 1;
    }
    return n;
}
static void put_symbol(bw_t* w, const huff_t* h, int s) { put_bits(w, h->code[s], h->len[s]); }
static void put_value(bw_t* w, int v, int nb) { /* negative values as v - 1 in nb bits */
    if (nb) put_bits(w, (unsigned)(v < 0 ? v - 1 : v) & ((1u << nb) - 1u), nb);
}

/* one component block: 64 FP32 samples (row-major, level-shifted) -> the
   quantised coefficients in row-major order */
static void block_coeffs(const float f[64], const float M[64], const float rq[64], int q[64]) {
    float t[64], F[64];
    for (int r = 0; r < 8; ++r) /* over the columns of each row */
        for (int l = 0; l < 8; ++l) {
            float acc = 0.0f;
            for (int c = 0; c < 8; ++c) acc = fmaf(f[r * 8 + c], M[l * 8 + c], acc);
            t[r * 8 + l] = acc;
        }
    for (int k = 0; k < 8; ++k) /* then over the rows */
        for (int l = 0; l < 8; ++l) {
            float acc = 0.0f;
            for (int r = 0; r < 8; ++r) acc = fmaf(M[k * 8 + r], t[r * 8 + l], acc);
            F[k * 8 + l] = acc;
        }
    for (int i = 0; i < 64; ++i) {
        const float x = F[i] * rq[i];
        int v = (int)truncf(x + copysignf(0.5f, x));
        if (i > 0) v = v > 1023 ? 1023 : (v < -1023 ? -1023 : v);
        q[i] = v;
    }
}

/* Encodes W x H RGB8 (row-major, 3 bytes per pixel) at `quality`; writes at
   most cap bytes to out and returns the full length. */
int64_t orc_jpeg(const uint8_t* rgb, int W, int H, int quality, uint8_t* out, int64_t cap) {
    int zz[64];
    zigzag(zz);
    uint8_t qt[2][64];
    orc_jpeg_qtable(quality, 0, qt[0]);
    orc_jpeg_qtable(quality, 1, qt[1]);
    float rq[2][64], M[64];
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 64; ++i) rq[c][i] = 1.0f / (float)qt[c][i];
    for (int k = 0; k < 8; ++k)
        for (int n = 0; n < 8; ++n) {
            const double ck = k == 0 ? sqrt(0.5) : 1.0;
            M[k * 8 + n] = (float)(0.5 * ck * cos((2 * n + 1) * k * M_PI / 16.0));
        }
    huff_t hdc[2], hac[2];
    huff_build(DCL_N, DC_SYM, &hdc[0]);
    huff_build(ACL_N, ACL_SYM, &hac[0]);
    huff_build(DCC_N, DC_SYM, &hdc[1]);
    huff_build(ACC_N, ACC_SYM, &hac[1]);

    bw_t w = {out, cap, 0, 0u, 0};
    const int W8 = (W + 7) / 8, H8 = (H + 7) / 8;
    /* SOI, APP0 (JFIF 1.01, no density units, no thumbnail) */
    put16(&w, 0xFFD8);
    put16(&w, 0xFFE0);
    put16(&w, 16);
    const uint8_t jfif[14] = {'J', 'F', 'I', 'F', 0, 1, 1, 0, 0, 1, 0, 1, 0, 0};
    for (int i = 0; i < 14; ++i) put_byte(&w, jfif[i]);
    /* DQT: both tables, 8-bit, in zig-zag order */
    put16(&w, 0xFFDB);
    put16(&w, 2 + 2 * 65);
    for (int c = 0; c < 2; ++c) {
        put_byte(&w, (uint8_t)c);
        for (int i = 0; i < 64; ++i) put_byte(&w, qt[c][zz[i]]);
    }
    /* SOF0: 8-bit, H x W, three components, 1x1 sampling, tables 0/1/1 */
    put16(&w, 0xFFC0);
    put16(&w, 17);
    put_byte(&w, 8);
    put16(&w, (unsigned)H);
    put16(&w, (unsigned)W);
    put_byte(&w, 3);
    for (int c = 0; c < 3; ++c) {
        put_byte(&w, (uint8_t)(c + 1));
        put_byte(&w, 0x11);
        put_byte(&w, (uint8_t)(c ? 1 : 0));
    }
    /* DHT: DC0, AC0, DC1, AC1 */
    {
        const uint8_t cls_id[4] = {0x00, 0x10, 0x01, 0x11};
        const int tab[4] = {0, 1, 2, 3};
        int len = 2;
        uint8_t n[16], s[162];
        for (int t = 0; t < 4; ++t) len += 17 + orc_jpeg_htable(tab[t], n, s);
        put16(&w, 0xFFC4);
        put16(&w, (unsigned)len);
        for (int t = 0; t < 4; ++t) {
            const int m = orc_jpeg_htable(tab[t], n, s);
            put_byte(&w, cls_id[t]);
            for (int i = 0; i < 16; ++i) put_byte(&w, n[i]);
            for (int i = 0; i < m; ++i) put_byte(&w, s[i]);
        }
    }
    /* DRI: 40 MCUs per interval */
    put16(&w, 0xFFDD);
    put16(&w, 4);
    put16(&w, ORC_RESTART_MCUS);
    /* SOS: three components, full spectral range */
    put16(&w, 0xFFDA);
    put16(&w, 12);
    put_byte(&w, 3);
    for (int c = 0; c < 3; ++c) {
        put_byte(&w, (uint8_t)(c + 1));
        put_byte(&w, c ? 0x11 : 0x00);
    }
    put_byte(&w, 0);
    put_byte(&w, 63);
    put_byte(&w, 0);

    int pred[3] = {0, 0, 0};
    const int64_t n_mcu = (int64_t)W8 * H8;
    for (int64_t m = 0; m < n_mcu; ++m) {
        if (m > 0 && m % ORC_RESTART_MCUS == 0) { /* end of an interval */
            pad_ones(&w);
            put16(&w, 0xFFD0u + (unsigned)((m / ORC_RESTART_MCUS - 1) % 8));
            pred[0] = pred[1] = pred[2] = 0;
        }
        const int by = (int)(m / W8), bx = (int)(m % W8);
        {
            for (int comp = 0; comp < 3; ++comp) {
                float f[64];
                for (int r = 0; r < 8; ++r)
                    for (int c = 0; c < 8; ++c) {
                        const int y = by * 8 + r < H ? by * 8 + r : H - 1;
                        const int x = bx * 8 + c < W ? bx * 8 + c : W - 1;
                        const uint8_t* p = rgb + ((int64_t)y * W + x) * 3;
                        const float R = (float)p[0], G = (float)p[1], B = (float)p[2];
                        float v;
                        if (comp == 0) v = fmaf(0.114f, B, fmaf(0.587f, G, 0.299f * R)) - 128.0f;
                        else if (comp == 1) v = fmaf(0.5f, B, fmaf(-0.331264f, G, -0.168736f * R));
                        else v = fmaf(-0.081312f, B, fmaf(-0.418688f, G, 0.5f * R));
                        f[r * 8 + c] = v;
                    }
                int q[64];
                block_coeffs(f, M, rq[comp ? 1 : 0], q);
                const huff_t* hd = &hdc[comp ? 1 : 0];
                const huff_t* ha = &hac[comp ? 1 : 0];
                const int diff = q[0] - pred[comp];
                pred[comp] = q[0];
                const int nd = magnitude_bits(diff);
                put_symbol(&w, hd, nd);
                put_value(&w, diff, nd);
                int run = 0;
                for (int i = 1; i < 64; ++i) {
                    const int v = q[zz[i]];
                    if (v == 0) {
                        ++run;
                        continue;
                    }
                    while (run > 15) {
                        put_symbol(&w, ha, 0xF0);
                        run -= 16;
                    }
                    const int nb = magnitude_bits(v);
                    put_symbol(&w, ha, (run << 4) | nb);
                    put_value(&w, v, nb);
                    run = 0;
                }
                if (run > 0) put_symbol(&w, ha, 0x00);
            }
        }
    }
    pad_ones(&w);
    put16(&w, 0xFFD9);
    return w.n;
}

/* The quantised coefficients of every block (MCU order: row of MCUs, then
   Y, Cb, Cr), row-major within a block; for the pins. */
void orc_jpeg_coeffs(const uint8_t* rgb, int W, int H, int quality, int32_t* out) {
    uint8_t qt[2][64];
    orc_jpeg_qtable(quality, 0, qt[0]);
    orc_jpeg_qtable(quality, 1, qt[1]);
    float rq[2][64], M[64];
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 64; ++i) rq[c][i] = 1.0f / (float)qt[c][i];
    for (int k = 0; k < 8; ++k)
        for (int n = 0; n < 8; ++n) {
            const double ck = k == 0 ? sqrt(0.5) : 1.0;
            M[k * 8 + n] = (float)(0.5 * ck * cos((2 * n + 1) * k * M_PI / 16.0));
        }
    const int W8 = (W + 7) / 8, H8 = (H + 7) / 8;
    int64_t b = 0;
    for (int by = 0; by < H8; ++by)
        for (int bx = 0; bx < W8; ++bx)
            for (int comp = 0; comp < 3; ++comp, ++b) {
                float f[64];
                for (int r = 0; r < 8; ++r)
                    for (int c = 0; c < 8; ++c) {
                        const int y = by * 8 + r < H ? by * 8 + r : H - 1;
                        const int x = bx * 8 + c < W ? bx * 8 + c : W - 1;
                        const uint8_t* p = rgb + ((int64_t)y * W + x) * 3;
                        const float R = (float)p[0], G = (float)p[1], B = (float)p[2];
                        float v;
                        if (comp == 0) v = fmaf(0.114f, B, fmaf(0.587f, G, 0.299f * R)) - 128.0f;
                        else if (comp == 1) v = fmaf(0.5f, B, fmaf(-0.331264f, G, -0.168736f * R));
                        else v = fmaf(-0.081312f, B, fmaf(-0.418688f, G, 0.5f * R));
                        f[r * 8 + c] = v;
                    }
                block_coeffs(f, M, rq[comp ? 1 : 0], out + b * 64);
            }
}

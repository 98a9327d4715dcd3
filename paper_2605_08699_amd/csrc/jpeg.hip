// Baseline JPEG encoder for CDNA4 (gfx950): the per-frame payload of the
// paper's backend (Section 5.1, Rendering Engine: frames leave as 8-bit JPEG;
// Sections 4.2 and 5.2: one stateless JPEG per request; Table 1 pairs each
// resolution of the bitrate ladder with a quality factor).
//
//   k_jpeg_seg    one workgroup per restart interval (40 MCUs in raster
//                 order, one thread per 8x8 block): colour transform, forward
//                 DCT and quantisation into LDS, the entropy-coded length of each block
//                 (DC prediction inside the interval), a workgroup scan of
//                 those lengths, then each block's Huffman codes ORed into the
//                 interval's bit buffer at its offset
//   k_jpeg_count  per interval: bytes after padding with 1-bits, plus one
//                 0x00 for every 0xFF byte, plus the restart marker
//   k_jpeg_pack   per interval: output offset = header + the intervals before
//                 it; the bytes with stuffing, the RSTn marker (EOI after the
//                 last); clears the consumed bit-buffer words for the next call
//
// Format choices (the standard leaves them open; the JPEG oracle makes the
// same ones): JFIF full-range YCbCr, 4:4:4, orthonormal DCT-II as two FP32
// FMA chains (columns of each row first, then rows), quantisation
// x = F (1/Q), q = trunc(x + copysign(1/2, x)), AC clamped to +-1023, the
// Annex K tables scaled by quality, restart intervals of 40 MCUs.
#include "tigas_internal.h"

namespace tigas {

namespace {

// Row-major index -> zig-zag scan position (Figure A.6), built by walking the
// anti-diagonals: upwards on even ones, downwards on odd ones.
struct ZigZag {
    uint8_t pos[64];
    constexpr ZigZag() : pos{} {
        int i = 0;
        for (int d = 0; d < 15; ++d) {
            const int hi = d < 8 ? d : 7, lo = d < 8 ? 0 : d - 7;
            for (int j = hi; j >= lo; --j) {
                const int row = (d & 1) ? d - j : j;
                pos[row * 8 + (d - row)] = (uint8_t)i++;
            }
        }
    }
};
__constant__ ZigZag kZigZag = ZigZag();

__device__ __forceinline__ int magnitude_bits(int v) { return 32 - __clz(v < 0 ? -v : v); }

// Bit counter and bit writer with one interface: put(value, nbits), value
// holding exactly nbits bits, most significant first.
struct BitCount {
    uint32_t n = 0;
    __device__ void put(uint32_t, int nb) { n += (uint32_t)nb; }
};
struct BitWrite {
    uint32_t* buf;  // the interval's words, stream bit i at bit 31 - i % 32 of word i / 32
    uint64_t acc;   // pending bits, left-aligned
    int n;          // pending bit count
    uint32_t w;     // word the pending bits start in
    __device__ BitWrite(uint32_t* b, uint32_t start) : buf(b), acc(0), n((int)(start & 31u)), w(start >> 5) {}
    __device__ void put(uint32_t v, int nb) {  // nb <= 27, so one word at most becomes full
        acc |= (uint64_t)v << (64 - n - nb);
        n += nb;
        if (n >= 32) {
            atomicOr(&buf[w], (uint32_t)(acc >> 32));  // a word may be shared with the neighbouring block
            acc <<= 32;
            n -= 32;
            ++w;
        }
    }
    __device__ void flush() {
        if (n > 0) atomicOr(&buf[w], (uint32_t)(acc >> 32));
    }
};

template <class S>
__device__ __forceinline__ void put_symbol(S& s, const uint32_t* h, int sym) {
    const uint32_t e = h[sym];  // length << 16 | code
    s.put(e & 0xffffu, (int)(e >> 16));
}
template <class S>
__device__ __forceinline__ void put_value(S& s, int v, int nb) {  // negative values as v - 1 in nb bits
    if (nb) s.put((uint32_t)(v < 0 ? v - 1 : v) & ((1u << nb) - 1u), nb);
}

// Entropy coding of one block (Annex F): DC difference category and bits,
// then AC run/size symbols with ZRL for 16 zeros and EOB before trailing zeros.
// nz has bit i set when scan position i holds a non-zero value, so the loop
// visits the non-zero AC values only (the runs are the gaps between them).
template <class S>
__device__ void code_block(const int16_t* zq, uint64_t nz, int pred, const uint32_t* hdc, const uint32_t* hac,
                           S& s) {
    const int diff = zq[0] - pred;
    const int nd = magnitude_bits(diff);
    put_symbol(s, hdc, nd);
    put_value(s, diff, nd);
    int prev = 0;
    for (uint64_t m = nz & ~1ull; m; m &= m - 1) {
        const int i = __builtin_ctzll(m);
        int run = i - prev - 1;
        while (run > 15) {
            put_symbol(s, hac, 0xF0);
            run -= 16;
        }
        const int v = zq[i];
        const int nb = magnitude_bits(v);
        put_symbol(s, hac, (run << 4) | nb);
        put_value(s, v, nb);
        prev = i;
    }
    if (prev < 63) put_symbol(s, hac, 0x00);
}

// Workgroup exclusive scan (JPEG_THREADS threads) through LDS.
__device__ uint32_t wg_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int d = 1; d < JPEG_THREADS; d <<= 1) {
        const uint32_t add = t >= d ? lds[t - d] : 0u;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const uint32_t incl = lds[t];
    *total = lds[JPEG_THREADS - 1];
    __syncthreads();
    return incl - v;
}

__device__ __forceinline__ uint32_t row_byte(const uint32_t* buf, uint32_t j, uint32_t bits) {
    uint32_t b = (buf[j >> 2] >> (24 - 8 * (j & 3u))) & 0xffu;
    const uint32_t used = bits - 8 * j;  // bits of this byte that belong to the stream
    if (used < 8) b |= 0xffu >> used;   // pad bits are ones
    return b;
}

}  // namespace

__global__ __launch_bounds__(JPEG_THREADS) void k_jpeg_seg(JpegArgs a) {
    static_assert(3 * JPEG_SEG_MCUS <= JPEG_THREADS, "one thread per block of an interval");
    // quantised coefficients of the interval in zig-zag order, one block per
    // thread; rows of 66 halves (33 words) so that the 64 lanes reading
    // coefficient i of their blocks meet in different LDS banks
    constexpr int ZS = 66;
    __shared__ int16_t s_coef[3 * JPEG_SEG_MCUS * ZS];
    __shared__ int32_t s_dc[3 * JPEG_SEG_MCUS];
    __shared__ uint64_t s_nz[3 * JPEG_SEG_MCUS];  // non-zero scan positions of each block
    __shared__ uint32_t s_huff[4 * 256];
    __shared__ uint32_t s_scan[JPEG_THREADS];
    __shared__ uint8_t s_pix[JPEG_SEG_MCUS * 64 * 3];  // the interval's 8x8 pixel blocks, edges repeated
    const int seg = blockIdx.x, t = threadIdx.x;
    const int64_t m0 = (int64_t)seg * JPEG_SEG_MCUS;
    const int nm = (int)min((int64_t)JPEG_SEG_MCUS, a.n_mcu - m0);
    const int nb = 3 * nm;
    for (int i = t; i < 4 * 256; i += JPEG_THREADS) s_huff[i] = a.huff[i];
    // the pixels of the interval, staged once: consecutive threads read
    // consecutive pixels of a block row (the three component threads of an
    // MCU share them)
    for (int i = t; i < nm * 64; i += JPEG_THREADS) {
        const int64_t mcu = m0 + i / 64;
        const int x = min((int)(mcu % a.w8) * 8 + (i & 7), a.width - 1);
        const int y = min((int)(mcu / a.w8) * 8 + ((i >> 3) & 7), a.height - 1);
        const uint8_t* p = a.rgb + ((size_t)y * a.width + x) * 3;
        s_pix[3 * i] = p[0];
        s_pix[3 * i + 1] = p[1];
        s_pix[3 * i + 2] = p[2];
    }
    __syncthreads();
    int16_t* zq = s_coef + (t < 3 * JPEG_SEG_MCUS ? t : 0) * ZS;
    const int comp = t % 3;

    // transform and quantise block t (Y, Cb, Cr of each MCU)
    if (t < nb) {
        const uint8_t* px = s_pix + (t / 3) * 64 * 3;
        float tr[64];  // rows transformed along x: tr[r][l]
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            float f[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const uint8_t* p = px + (r * 8 + c) * 3;
                const float R = (float)p[0], G = (float)p[1], B = (float)p[2];
                float v;
                if (comp == 0) v = __builtin_fmaf(0.114f, B, __builtin_fmaf(0.587f, G, 0.299f * R)) - 128.0f;
                else if (comp == 1) v = __builtin_fmaf(0.5f, B, __builtin_fmaf(-0.331264f, G, -0.168736f * R));
                else v = __builtin_fmaf(-0.081312f, B, __builtin_fmaf(-0.418688f, G, 0.5f * R));
                f[c] = v;
            }
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                float acc = 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) acc = __builtin_fmaf(f[c], a.dct[l * 8 + c], acc);
                tr[r * 8 + l] = acc;
            }
        }
        const float* rq = comp ? a.rq_chroma : a.rq_luma;
        uint64_t nz = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                float acc = 0.0f;
#pragma unroll
                for (int r = 0; r < 8; ++r) acc = __builtin_fmaf(a.dct[k * 8 + r], tr[r * 8 + l], acc);
                const float x = acc * rq[k * 8 + l];
                int v = (int)__builtin_truncf(x + __builtin_copysignf(0.5f, x));
                if (k + l > 0) v = max(-1023, min(1023, v));
                const int p = kZigZag.pos[k * 8 + l];
                zq[p] = (int16_t)v;
                nz |= v != 0 ? 1ull << p : 0ull;
                if (k + l == 0) s_dc[t] = v;
            }
        s_nz[t] = nz;
    }
    __syncthreads();

    // entropy-coded length of the block; DC predicted from the previous block
    // of the same component in the interval (the interval starts at zero)
    const uint32_t* hdc = s_huff + (comp ? 512 : 0);
    const uint32_t* hac = s_huff + (comp ? 768 : 256);
    const int pred = t >= 3 && t < nb ? s_dc[t - 3] : 0;
    uint32_t len = 0;
    if (t < nb) {
        BitCount c;
        code_block(zq, s_nz[t], pred, hdc, hac, c);  // this thread's own block
        len = c.n;
    }
    uint32_t total;
    const uint32_t off = wg_excl_scan(len, s_scan, &total);
    if (t == 0) a.seg_bits[seg] = total;

    // the codes, ORed into the (cleared) bit buffer of the interval
    if (t < nb) {
        BitWrite w(a.bits + (size_t)seg * a.seg_words, off);
        code_block(zq, s_nz[t], pred, hdc, hac, w);
        w.flush();
    }
}

__global__ __launch_bounds__(JPEG_THREADS) void k_jpeg_count(JpegArgs a) {
    __shared__ uint32_t s_scan[JPEG_THREADS];
    const int seg = blockIdx.x;
    const uint32_t bits = a.seg_bits[seg];
    const uint32_t nbytes = (bits + 7) / 8;
    const uint32_t* buf = a.bits + (size_t)seg * a.seg_words;
    uint32_t ff = 0;
    for (uint32_t j = threadIdx.x; j < nbytes; j += JPEG_THREADS) ff += row_byte(buf, j, bits) == 0xffu ? 1u : 0u;
    uint32_t total;
    wg_excl_scan(ff, s_scan, &total);
    if (threadIdx.x == 0) a.seg_len[seg] = nbytes + total + (seg + 1 < a.nseg ? 2u : 0u);
}

__global__ __launch_bounds__(JPEG_THREADS) void k_jpeg_pack(JpegArgs a) {
    __shared__ uint32_t s_scan[JPEG_THREADS];
    const int seg = blockIdx.x, t = threadIdx.x;
    // output offset of the interval: the header and every interval before it
    uint32_t before = 0;
    for (int r = t; r < seg; r += JPEG_THREADS) before += a.seg_len[r];
    uint32_t tot_before;
    wg_excl_scan(before, s_scan, &tot_before);
    const uint64_t base = a.header_len + (uint64_t)tot_before;
    const uint32_t bits = a.seg_bits[seg];
    const uint32_t nbytes = (bits + 7) / 8;
    uint32_t* buf = a.bits + (size_t)seg * a.seg_words;
    // a contiguous run of bytes per thread; its 0xFF count places it
    const uint32_t per = (nbytes + JPEG_THREADS - 1) / JPEG_THREADS;
    const uint32_t j0 = min(nbytes, (uint32_t)t * per), j1 = min(nbytes, j0 + per);
    uint32_t ff = 0;
    for (uint32_t j = j0; j < j1; ++j) ff += row_byte(buf, j, bits) == 0xffu ? 1u : 0u;
    uint32_t ff_total;
    const uint32_t ff_before = wg_excl_scan(ff, s_scan, &ff_total);
    uint64_t pos = base + j0 + ff_before;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t v = row_byte(buf, j, bits);
        if (pos < a.capacity) a.out[pos] = (uint8_t)v;
        ++pos;
        if (v == 0xffu) {
            if (pos < a.capacity) a.out[pos] = 0;
            ++pos;
        }
    }
    const uint64_t end = base + nbytes + ff_total;
    if (t == 0) {
        const bool last = seg + 1 == a.nseg;
        const uint8_t m = last ? 0xD9 : (uint8_t)(0xD0 + (seg & 7));  // RSTn, or EOI after the last interval
        if (end < a.capacity) a.out[end] = 0xFF;
        if (end + 1 < a.capacity) a.out[end + 1] = m;
        if (last) *a.out_len = end + 2;
    }
    __syncthreads();
    // leave the bit buffer cleared for the next call
    for (uint32_t i = t; i < (bits + 31) / 32; i += JPEG_THREADS) buf[i] = 0u;
}

#define TIGAS_JPEG_LAUNCH(kernel, grid, st, a)                                    \
    do {                                                                          \
        KernelTimer* kt_ = g_kernel_timer;                                        \
        if (kt_) kt_->before(reinterpret_cast<const void*>(kernel), st);         \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(JPEG_THREADS), 0, st, a);     \
        if (kt_) kt_->after(st);                                                  \
    } while (0)

void launch_jpeg(const JpegArgs& a, hipStream_t st) {
    TIGAS_JPEG_LAUNCH(k_jpeg_seg, a.nseg, st, a);
    TIGAS_JPEG_LAUNCH(k_jpeg_count, a.nseg, st, a);
    TIGAS_JPEG_LAUNCH(k_jpeg_pack, a.nseg, st, a);
}

}  // namespace tigas

/*
 * fk_oracle.c -- plain CPU oracle for the fused preprocessing chain.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the GPU library never
 * includes, links or calls anything here, and this file includes nothing of
 * the GPU library.
 *
 * What it computes.  Fusion changes where intermediates live, not what is
 * computed (Section II: the fused kernel performs exactly the operations of
 * the separate kernels, keeping intermediates in registers instead of
 * DRAM).  So the oracle is the plain definition: each operation of the chain
 * runs UNFUSED, as one full pass over the whole image, and every
 * intermediate is stored as fp32 -- the separate-kernel pipeline of the
 * kernel-call algorithm and of the vertical-fusion figure (part A), whose
 * intermediate images are float buffers (Section VI-L names crop_32F and the
 * resized buffer).
 *
 * Next to the fp32 result it carries, per element, an fp64 shadow of the
 * same operation sequence (each op rounded to fp64, never to fp32) and the largest
 * magnitude the element took along the chain; tests use both to bound
 * rounding error.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - Resize (Sections VI-F, VI-J name "Resize" only): bilinear, half-pixel
 *    centres, no antialiasing, taps clamped to the crop; source coordinate
 *    sx = max(fma(ox + 0.5, w / OW, -0.5), 0) in fp32, x0 = floor(sx),
 *    x1 = min(x0 + 1, w - 1), ax = sx - x0; two horizontal lerps and one
 *    vertical lerp, each written as fma(a, p1 - p0, p0); the result stays
 *    fp32 (not re-quantised).
 *  - Values: u8 and fp16 sources convert to fp32 exactly, and every
 *    arithmetic op runs in fp32, so the running value is held as fp32 from
 *    the read onwards; "cvt" is then numerically the identity.
 *  - Nearest resize (the other interpolation): output index o takes source
 *    index floor((2o + 1) * in / (2 * out)) in exact integer arithmetic, the
 *    source pixel whose extent holds the output pixel's centre (a centre on
 *    a pixel boundary goes to the higher index).
 *  - NV12 read: the frame is a W x H luma plane followed, at the same pitch,
 *    by H/2 rows of W/2 interleaved (U, V) pairs (W and H even).  Pixel
 *    (x, y) takes Y[y][x] and the chroma pair of (x/2, y/2) (each pair
 *    serves a 2 x 2 block) and becomes three fp32 values in B, G, R order by
 *    the ITU-R BT.601 limited-range matrix: with y' = Y - 16, u = U - 128,
 *    v = V - 128 and c = 1.164 y', B = c + 2.018 u, G = (c - 0.813 v) -
 *    0.391 u, R = c + 1.596 v, every product and sum one fp32 operation in
 *    that order.  The ROI is in luma pixels; the NV12 resize read applies
 *    the bilinear resize above to the converted crop.
 *  - Swap (ColorConvert BGR->RGB): exchanges channels 0 and 2; channel 3 is
 *    kept; a no-op for one channel.  Per-channel constants index channels by
 *    their position after earlier swaps.
 *  - Mul/Add/Sub/Div: one IEEE fp32 operation each (round to nearest even),
 *    no contraction; Div is a true division.
 *  - Write: packed out[(y*W + x)*C + c] or planar out[(c*H + y)*W + x];
 *    fp16 outputs round to nearest even.
 *  - Stats write (the reduction pattern of Section IV-C: several reductions
 *    of one matrix from a single read): instead of an image, each item's
 *    output is, per channel c, {min, max, sum, mean} of the chain's fp32
 *    values, as four doubles at dst[4c .. 4c+3].  min and max are IEEE
 *    minNum/maxNum over the values in row-major order (a NaN value is
 *    skipped); sum adds the values converted to fp64 in row-major order;
 *    mean = sum / (number of pixels), in fp64.
 *  - Double-precision chains (the data-type experiment of Section VI-I
 *    names float->double and double->double, whose kernels compute in
 *    double): a chain whose write is fp64 (packed or planar) runs in fp64
 *    from the read on.  The read takes u8, fp16 and fp32 elements exactly
 *    and fp64 elements as they are; the cast is the identity; every
 *    Mul/Add/Sub/Div is one IEEE fp64 operation with the op's fp32 constant
 *    taken exactly as a double; the write stores the fp64 value.  Only the
 *    plain read takes such chains, and an fp64 frame only with an fp64
 *    write.  The fp64 value held next to each fp32 value (below) is that
 *    chain: it already rounds every op to fp64.
 *  - Loop (the repeat op of Section VI-B, which applies one op many times
 *    without spending kernel parameters on each copy): the `span` ops just
 *    before it run `count` times in all, in order, before the chain goes
 *    on.  Its body holds Mul/Add/Sub/Div ops only, so a loop neither
 *    crosses a swap nor contains another loop.
 *
 * Build: gcc -O2 -std=c11 -fno-fast-math -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_U8 = 0, ORC_F16 = 1, ORC_F32 = 2, ORC_F64 = 3 };
enum {
    ORC_READ_PLAIN = 0,
    ORC_READ_CROP_RESIZE = 1,
    ORC_READ_CROP_NEAREST = 2,
    ORC_READ_NV12 = 3,
    ORC_READ_NV12_RESIZE = 4,
};
enum { ORC_SWAP = 0, ORC_CVT = 1, ORC_MUL = 2, ORC_ADD = 3, ORC_SUB = 4, ORC_DIV = 5, ORC_LOOP = 6 };
enum { ORC_PACKED = 0, ORC_PLANAR = 1, ORC_STATS = 2 };

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ENOMEM = -3,
};

typedef struct {
    int32_t kind;
    int32_t nconst; /* 0, 1 (scalar) or C (one per channel) */
    float k[4];
    int32_t span;   /* ORC_LOOP: number of ops just before it that repeat */
    int32_t count;  /* ORC_LOOP: how many times they run in all (>= 1) */
} orc_op;

typedef struct {
    int32_t read_kind;
    int32_t in_dtype;
    int32_t channels;
    const orc_op *ops;
    int32_t n_ops;
    int32_t out_dtype; /* ORC_F32 or ORC_F16; ORC_F64 with ORC_STATS, or with a
                          plain read for a double-precision chain */
    int32_t layout;    /* ORC_PACKED, ORC_PLANAR or ORC_STATS */
} orc_chain;

typedef struct {
    const void *src;     /* packed HWC frame, host memory */
    int32_t W, H;        /* frame size in pixels */
    int64_t pitch;       /* bytes between frame rows */
    int32_t x, y, w, h;  /* region of interest */
    int32_t ow, oh;      /* output size (crop+resize); plain read uses w, h */
    void *dst;           /* output image in the chain's output dtype/layout,
                            or 4 * channels doubles for ORC_STATS */
    double *v64;         /* optional: fp64 shadow, same layout as dst (images only) */
    float *smax;         /* optional: largest |value| along the chain (images only) */
} orc_item;

/* ---------------------------------------------------------------- fp16 -- */

/* IEEE binary16 -> binary32; exact for every input. */
float orc_half_to_float(uint16_t h)
{
    uint32_t sign = (uint32_t)(h >> 15) & 1u;
    int32_t exp = (h >> 10) & 0x1f;
    uint32_t man = h & 0x3ffu;
    float mag;
    if (exp == 0) {
        mag = ldexpf((float)man, -24); /* subnormal (or zero) */
    } else if (exp == 31) {
        mag = man ? NAN : INFINITY;
    } else {
        mag = ldexpf((float)(man | 0x400u), exp - 25);
    }
    return sign ? -mag : mag;
}

/* binary32 -> binary16, round to nearest, ties to even. */
uint16_t orc_float_to_half(float f)
{
    uint32_t bits;
    memcpy(&bits, &f, sizeof bits);
    uint16_t sign = (uint16_t)((bits >> 16) & 0x8000u);
    if (isnan(f))
        return (uint16_t)(sign | 0x7e00u);
    double a = fabs((double)f);
    if (a >= 65520.0) /* halfway between 65504 and 2^16 rounds to inf */
        return (uint16_t)(sign | 0x7c00u);
    /* Scale so the binary16 unit in the last place becomes 1, then round to
     * an integer with ties to even (nearbyint in the default mode). */
    int e;
    frexp(a, &e); /* a = m * 2^e, m in [0.5, 1) */
    int ulp_exp = e - 11;  /* normal numbers: 11 significant bits */
    if (ulp_exp < -24)
        ulp_exp = -24;     /* subnormal spacing */
    double q = nearbyint(ldexp(a, -ulp_exp)); /* exact scaling, RNE */
    double r = ldexp(q, ulp_exp);
    if (r >= 65520.0)
        return (uint16_t)(sign | 0x7c00u);
    if (r == 0.0)
        return sign;
    /* Re-encode r, which is exactly representable in binary16. */
    int re;
    double rm = frexp(r, &re); /* r = rm * 2^re */
    int biased = re - 1 + 15;
    uint16_t out;
    if (biased <= 0) {
        out = (uint16_t)ldexp(r, 24); /* subnormal: multiple of 2^-24 */
    } else {
        uint16_t mant = (uint16_t)(ldexp(rm, 11) - 1024.0);
        out = (uint16_t)((biased << 10) | mant);
    }
    return (uint16_t)(sign | out);
}

/* ----------------------------------------------------------- elements -- */

static size_t dtype_size(int32_t dt)
{
    return dt == ORC_U8 ? 1u : dt == ORC_F16 ? 2u : dt == ORC_F64 ? 8u : 4u;
}

/* Element (x, y, c) of a packed fp64 frame. */
static double frame_elem64(const orc_item *it, int32_t C, int32_t x, int32_t y, int32_t c)
{
    const uint8_t *row = (const uint8_t *)it->src + (int64_t)y * it->pitch;
    double v;
    memcpy(&v, row + ((size_t)x * (size_t)C + (size_t)c) * 8, 8);
    return v;
}

/* Element (x, y, c) of a packed HWC frame, converted to fp32 (exact). */
static float frame_elem(const orc_item *it, int32_t dt, int32_t C, int32_t x, int32_t y,
                        int32_t c)
{
    const uint8_t *row = (const uint8_t *)it->src + (int64_t)y * it->pitch;
    size_t idx = (size_t)x * (size_t)C + (size_t)c;
    if (dt == ORC_U8)
        return (float)row[idx];
    if (dt == ORC_F16) {
        uint16_t h;
        memcpy(&h, row + idx * 2, 2);
        return orc_half_to_float(h);
    }
    float v;
    memcpy(&v, row + idx * 4, 4);
    return v;
}

/* One intermediate image: packed HWC, fp32 value, fp64 shadow, running max. */
typedef struct {
    int32_t w, h, C;
    float *v;
    double *d;
    float *s;
} img;

static int img_alloc(img *m, int32_t w, int32_t h, int32_t C)
{
    size_t n = (size_t)w * (size_t)h * (size_t)C;
    m->w = w;
    m->h = h;
    m->C = C;
    m->v = (float *)malloc(n * sizeof(float));
    m->d = (double *)malloc(n * sizeof(double));
    m->s = (float *)malloc(n * sizeof(float));
    if (!m->v || !m->d || !m->s)
        return ORC_ENOMEM;
    return ORC_OK;
}

static void img_free(img *m)
{
    free(m->v);
    free(m->d);
    free(m->s);
    m->v = NULL;
    m->d = NULL;
    m->s = NULL;
}

/* ------------------------------------------------------------- steps -- */

/* Crop: the region of interest becomes its own image (values to fp32). */
static int step_crop(const orc_chain *ch, const orc_item *it, img *out)
{
    int32_t C = ch->channels;
    int rc = img_alloc(out, it->w, it->h, C);
    if (rc)
        return rc;
    for (int32_t j = 0; j < it->h; ++j)
        for (int32_t i = 0; i < it->w; ++i)
            for (int32_t c = 0; c < C; ++c) {
                size_t o = ((size_t)j * (size_t)it->w + (size_t)i) * (size_t)C + (size_t)c;
                if (ch->in_dtype == ORC_F64) {
                    double d = frame_elem64(it, C, it->x + i, it->y + j, c);
                    out->v[o] = (float)d;
                    out->d[o] = d;
                    out->s[o] = fabsf((float)d);
                    continue;
                }
                float v = frame_elem(it, ch->in_dtype, C, it->x + i, it->y + j, c);
                out->v[o] = v;
                out->d[o] = (double)v;
                out->s[o] = fabsf(v);
            }
    return ORC_OK;
}

/* NV12 pixel (x, y) of the frame -> B, G, R (BT.601 limited range). */
static void nv12_bgr(const orc_item *it, int32_t x, int32_t y, float out[3])
{
    const uint8_t *base = (const uint8_t *)it->src;
    float Y = (float)base[(int64_t)y * it->pitch + x];
    const uint8_t *uv = base + ((int64_t)it->H + y / 2) * it->pitch + (int64_t)(x / 2) * 2;
    float u = (float)uv[0] - 128.0f;
    float v = (float)uv[1] - 128.0f;
    float c = 1.164f * (Y - 16.0f);
    out[0] = c + 2.018f * u;
    out[1] = (c - 0.813f * v) - 0.391f * u;
    out[2] = c + 1.596f * v;
}

/* NV12 crop: the region of interest, converted, becomes its own image. */
static int step_crop_nv12(const orc_item *it, img *out)
{
    int rc = img_alloc(out, it->w, it->h, 3);
    if (rc)
        return rc;
    for (int32_t j = 0; j < it->h; ++j)
        for (int32_t i = 0; i < it->w; ++i) {
            float bgr[3];
            nv12_bgr(it, it->x + i, it->y + j, bgr);
            for (int32_t c = 0; c < 3; ++c) {
                size_t o = ((size_t)j * (size_t)it->w + (size_t)i) * 3u + (size_t)c;
                out->v[o] = bgr[c];
                out->d[o] = (double)bgr[c];
                out->s[o] = fabsf(bgr[c]);
            }
        }
    return ORC_OK;
}

/* Nearest resize of a whole image to ow x oh. */
static int step_nearest(const img *in, int32_t ow, int32_t oh, img *out)
{
    int32_t C = in->C;
    int rc = img_alloc(out, ow, oh, C);
    if (rc)
        return rc;
    for (int32_t oy = 0; oy < oh; ++oy) {
        int64_t sy = ((int64_t)2 * oy + 1) * in->h / ((int64_t)2 * oh);
        for (int32_t ox = 0; ox < ow; ++ox) {
            int64_t sx = ((int64_t)2 * ox + 1) * in->w / ((int64_t)2 * ow);
            for (int32_t c = 0; c < C; ++c) {
                size_t i = ((size_t)sy * (size_t)in->w + (size_t)sx) * (size_t)C + (size_t)c;
                size_t o = ((size_t)oy * (size_t)ow + (size_t)ox) * (size_t)C + (size_t)c;
                out->v[o] = in->v[i];
                out->d[o] = in->d[i];
                out->s[o] = in->s[i];
            }
        }
    }
    return ORC_OK;
}

/* Source coordinate of output index o for a scale of in/out (half-pixel
 * centres), clamped below at 0; returns the two tap indices and weight. */
static void bilinear_coord(int32_t o, float scale, int32_t in_size, int32_t *i0, int32_t *i1,
                           float *a)
{
    float s = fmaf((float)o + 0.5f, scale, -0.5f);
    if (s < 0.0f)
        s = 0.0f;
    int32_t lo = (int32_t)floorf(s);
    if (lo > in_size - 1) /* cannot happen for in/out scales; kept as a guard */
        lo = in_size - 1;
    *i0 = lo;
    *i1 = lo + 1 < in_size ? lo + 1 : in_size - 1;
    *a = s - (float)lo;
}

/* Bilinear resize of a whole image to ow x oh. */
static int step_resize(const img *in, int32_t ow, int32_t oh, img *out)
{
    int32_t C = in->C;
    int rc = img_alloc(out, ow, oh, C);
    if (rc)
        return rc;
    float sx_scale = (float)in->w / (float)ow;
    float sy_scale = (float)in->h / (float)oh;
    for (int32_t oy = 0; oy < oh; ++oy) {
        int32_t y0, y1;
        float ay;
        bilinear_coord(oy, sy_scale, in->h, &y0, &y1, &ay);
        for (int32_t ox = 0; ox < ow; ++ox) {
            int32_t x0, x1;
            float ax;
            bilinear_coord(ox, sx_scale, in->w, &x0, &x1, &ax);
            for (int32_t c = 0; c < C; ++c) {
                size_t i00 = ((size_t)y0 * (size_t)in->w + (size_t)x0) * (size_t)C + (size_t)c;
                size_t i01 = ((size_t)y0 * (size_t)in->w + (size_t)x1) * (size_t)C + (size_t)c;
                size_t i10 = ((size_t)y1 * (size_t)in->w + (size_t)x0) * (size_t)C + (size_t)c;
                size_t i11 = ((size_t)y1 * (size_t)in->w + (size_t)x1) * (size_t)C + (size_t)c;
                float p00 = in->v[i00], p01 = in->v[i01], p10 = in->v[i10], p11 = in->v[i11];
                float top = fmaf(ax, p01 - p00, p00);
                float bot = fmaf(ax, p11 - p10, p10);
                float v = fmaf(ay, bot - top, top);
                double d00 = in->d[i00], d01 = in->d[i01], d10 = in->d[i10], d11 = in->d[i11];
                double dtop = d00 + (double)ax * (d01 - d00);
                double dbot = d10 + (double)ax * (d11 - d10);
                double dv = dtop + (double)ay * (dbot - dtop);
                float sm = in->s[i00];
                if (in->s[i01] > sm) sm = in->s[i01];
                if (in->s[i10] > sm) sm = in->s[i10];
                if (in->s[i11] > sm) sm = in->s[i11];
                if (fabsf(v) > sm) sm = fabsf(v);
                size_t o = ((size_t)oy * (size_t)ow + (size_t)ox) * (size_t)C + (size_t)c;
                out->v[o] = v;
                out->d[o] = dv;
                out->s[o] = sm;
            }
        }
    }
    return ORC_OK;
}

/* Swap channels 0 and 2 of every pixel (BGR <-> RGB); alpha untouched. */
static void step_swap(img *m)
{
    if (m->C < 3)
        return;
    size_t npix = (size_t)m->w * (size_t)m->h;
    for (size_t p = 0; p < npix; ++p) {
        size_t a = p * (size_t)m->C, b = a + 2;
        float tv = m->v[a];
        m->v[a] = m->v[b];
        m->v[b] = tv;
        double td = m->d[a];
        m->d[a] = m->d[b];
        m->d[b] = td;
        float ts = m->s[a];
        m->s[a] = m->s[b];
        m->s[b] = ts;
    }
}

/* One binary arithmetic op with a scalar or per-channel constant. */
static void step_arith(img *m, const orc_op *op)
{
    size_t npix = (size_t)m->w * (size_t)m->h;
    for (size_t p = 0; p < npix; ++p)
        for (int32_t c = 0; c < m->C; ++c) {
            size_t i = p * (size_t)m->C + (size_t)c;
            float k = op->nconst == 1 ? op->k[0] : op->k[c];
            float v = m->v[i];
            double d = m->d[i];
            float r;
            double rd;
            switch (op->kind) {
            case ORC_MUL: r = v * k; rd = d * (double)k; break;
            case ORC_ADD: r = v + k; rd = d + (double)k; break;
            case ORC_SUB: r = v - k; rd = d - (double)k; break;
            default:      r = v / k; rd = d / (double)k; break; /* ORC_DIV */
            }
            m->v[i] = r;
            m->d[i] = rd;
            if (fabsf(r) > m->s[i])
                m->s[i] = fabsf(r);
        }
}

/* Write the final image to the item's output in the chain's layout/dtype. */
static void step_write(const orc_chain *ch, const img *m, const orc_item *it)
{
    int32_t C = m->C;
    for (int32_t y = 0; y < m->h; ++y)
        for (int32_t x = 0; x < m->w; ++x)
            for (int32_t c = 0; c < C; ++c) {
                size_t i = ((size_t)y * (size_t)m->w + (size_t)x) * (size_t)C + (size_t)c;
                size_t o = ch->layout == ORC_PLANAR
                               ? ((size_t)c * (size_t)m->h + (size_t)y) * (size_t)m->w + (size_t)x
                               : i;
                if (ch->out_dtype == ORC_F16)
                    ((uint16_t *)it->dst)[o] = orc_float_to_half(m->v[i]);
                else if (ch->out_dtype == ORC_F64)
                    ((double *)it->dst)[o] = m->d[i];  /* the fp64 chain */
                else
                    ((float *)it->dst)[o] = m->v[i];
                if (it->v64)
                    it->v64[o] = m->d[i];
                if (it->smax)
                    it->smax[o] = m->s[i];
            }
}

/* Per-channel statistics of the final image (the stats write). */
static void step_stats(const img *m, const orc_item *it)
{
    int32_t C = m->C;
    size_t npix = (size_t)m->w * (size_t)m->h;
    double *out = (double *)it->dst;
    for (int32_t c = 0; c < C; ++c) {
        float mn = INFINITY, mx = -INFINITY;
        double sum = 0.0;
        for (size_t p = 0; p < npix; ++p) {
            float v = m->v[p * (size_t)C + (size_t)c];
            mn = fminf(mn, v);
            mx = fmaxf(mx, v);
            sum += (double)v;
        }
        out[4 * c + 0] = (double)mn;
        out[4 * c + 1] = (double)mx;
        out[4 * c + 2] = sum;
        out[4 * c + 3] = sum / (double)npix;
    }
}

/* ---------------------------------------------------------- validate -- */

static int chain_ok(const orc_chain *ch)
{
    if (!ch || (ch->n_ops > 0 && !ch->ops) || ch->n_ops < 0)
        return 0;
    if (ch->read_kind < ORC_READ_PLAIN || ch->read_kind > ORC_READ_NV12_RESIZE)
        return 0;
    if ((ch->read_kind == ORC_READ_NV12 || ch->read_kind == ORC_READ_NV12_RESIZE) &&
        (ch->in_dtype != ORC_U8 || ch->channels != 3))
        return 0;
    if (ch->in_dtype < ORC_U8 || ch->in_dtype > ORC_F64)
        return 0;
    if (ch->channels != 1 && ch->channels != 3 && ch->channels != 4)
        return 0;
    if (ch->layout == ORC_STATS) {
        if (ch->out_dtype != ORC_F64)
            return 0;
    } else {
        if (ch->out_dtype != ORC_F32 && ch->out_dtype != ORC_F16 && ch->out_dtype != ORC_F64)
            return 0;
        if (ch->layout != ORC_PACKED && ch->layout != ORC_PLANAR)
            return 0;
        /* double-precision chains: plain reads only */
        if (ch->out_dtype == ORC_F64 && ch->read_kind != ORC_READ_PLAIN)
            return 0;
    }
    /* an fp64 frame feeds a double-precision chain only */
    if (ch->in_dtype == ORC_F64 && (ch->layout == ORC_STATS || ch->out_dtype != ORC_F64))
        return 0;
    for (int32_t i = 0; i < ch->n_ops; ++i) {
        const orc_op *op = &ch->ops[i];
        if (op->kind < ORC_SWAP || op->kind > ORC_LOOP)
            return 0;
        if (op->kind == ORC_LOOP) {
            if (op->nconst != 0 || op->span < 1 || op->span > i || op->count < 1)
                return 0;
            for (int32_t j = i - op->span; j < i; ++j)
                if (ch->ops[j].kind < ORC_MUL || ch->ops[j].kind > ORC_DIV)
                    return 0;
        } else if (op->kind == ORC_SWAP || op->kind == ORC_CVT) {
            if (op->nconst != 0)
                return 0;
        } else if (op->nconst != 1 && op->nconst != ch->channels) {
            return 0;
        }
    }
    return 1;
}

static int item_ok(const orc_chain *ch, const orc_item *it)
{
    const int nv12 = ch->read_kind == ORC_READ_NV12 || ch->read_kind == ORC_READ_NV12_RESIZE;
    if (!it->src || !it->dst || it->W < 1 || it->H < 1)
        return 0;
    if (nv12 ? (it->pitch < it->W || it->W % 2 || it->H % 2)
             : it->pitch < (int64_t)it->W * ch->channels * (int64_t)dtype_size(ch->in_dtype))
        return 0;
    if (it->w < 1 || it->h < 1 || it->x < 0 || it->y < 0)
        return 0;
    if ((int64_t)it->x + it->w > it->W || (int64_t)it->y + it->h > it->H)
        return 0;
    if ((ch->read_kind == ORC_READ_CROP_RESIZE || ch->read_kind == ORC_READ_CROP_NEAREST ||
         ch->read_kind == ORC_READ_NV12_RESIZE) && (it->ow < 1 || it->oh < 1))
        return 0;
    return 1;
}

/* --------------------------------------------------------------- API -- */

int orc_validate(const orc_chain *ch, const orc_item *items, int32_t n)
{
    if (!chain_ok(ch) || n < 0 || (n > 0 && !items))
        return ORC_EINVAL;
    for (int32_t b = 0; b < n; ++b)
        if (!item_ok(ch, &items[b]))
            return ORC_EINVAL;
    return ORC_OK;
}

/* Run the chain, unfused, on each item in turn. */
int orc_run(const orc_chain *ch, const orc_item *items, int32_t n)
{
    int rc = orc_validate(ch, items, n);
    if (rc)
        return rc;
    for (int32_t b = 0; b < n; ++b) {
        const orc_item *it = &items[b];
        img cur = {0}, nxt = {0};
        if (ch->read_kind == ORC_READ_NV12 || ch->read_kind == ORC_READ_NV12_RESIZE)
            rc = step_crop_nv12(it, &cur);
        else
            rc = step_crop(ch, it, &cur);
        if (!rc && (ch->read_kind == ORC_READ_CROP_RESIZE || ch->read_kind == ORC_READ_NV12_RESIZE)) {
            rc = step_resize(&cur, it->ow, it->oh, &nxt);
            img_free(&cur);
            cur = nxt;
        } else if (!rc && ch->read_kind == ORC_READ_CROP_NEAREST) {
            rc = step_nearest(&cur, it->ow, it->oh, &nxt);
            img_free(&cur);
            cur = nxt;
        }
        for (int32_t i = 0; !rc && i < ch->n_ops; ++i) {
            const orc_op *op = &ch->ops[i];
            if (op->kind == ORC_SWAP)
                step_swap(&cur);
            else if (op->kind == ORC_CVT)
                ; /* fp32 conversion already exact at the read */
            else if (op->kind == ORC_LOOP)
                /* the body ran once on the way here: count - 1 more times */
                for (int32_t r = 1; r < op->count; ++r)
                    for (int32_t j = i - op->span; j < i; ++j)
                        step_arith(&cur, &ch->ops[j]);
            else
                step_arith(&cur, op);
        }
        if (!rc && ch->layout == ORC_STATS)
            step_stats(&cur, it);
        else if (!rc)
            step_write(ch, &cur, it);
        img_free(&cur);
        if (rc)
            return rc;
    }
    return ORC_OK;
}

/* Resize of one plane of fp32 values (used by the pins to test the resize
 * step in isolation, without the u8 read). */
int orc_resize_f32(const float *src, int32_t w, int32_t h, int32_t C, float *dst, int32_t ow,
                   int32_t oh)
{
    if (!src || !dst || w < 1 || h < 1 || ow < 1 || oh < 1 || C < 1)
        return ORC_EINVAL;
    img in = {0}, out = {0};
    int rc = img_alloc(&in, w, h, C);
    if (rc) {
        img_free(&in);
        return rc;
    }
    size_t n = (size_t)w * (size_t)h * (size_t)C;
    for (size_t i = 0; i < n; ++i) {
        in.v[i] = src[i];
        in.d[i] = (double)src[i];
        in.s[i] = fabsf(src[i]);
    }
    rc = step_resize(&in, ow, oh, &out);
    if (!rc)
        memcpy(dst, out.v, (size_t)ow * (size_t)oh * (size_t)C * sizeof(float));
    img_free(&in);
    img_free(&out);
    return rc;
}

/* fk_client.c -- a plain C11 consumer of libfkmi.so through include/fk.h
 * and the HIP runtime API: no Python, no torch.
 *
 * Runs the normalisation chain (crop + bilinear resize -> BGR->RGB -> fp32
 * -> x 1/255 -> - mean -> / std -> planar fp32) over a list of crops of one
 * packed HWC u8 BGR frame in one fused launch, and writes the planar fp32
 * outputs back to back.  Prints the chain's constants as hexadecimal floats
 * first, so a checker can rebuild the same chain.
 *
 * usage: fk_client FRAME_FILE WIDTH HEIGHT OUT_W OUT_H STRICT CROPS_FILE OUT_FILE
 *   FRAME_FILE: WIDTH * HEIGHT * 3 bytes; CROPS_FILE: lines "x y w h".
 * Exit status 0 on success, 1 on a usage or file error, 2 on a library or
 * HIP error (the message goes to stderr). */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "fk.h"

#define MAX_CROPS 4096

static int hip_ok(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return 1;
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 0;
}

static int fk_ok(fk_status s, const char *what)
{
    if (s == FK_OK)
        return 1;
    fprintf(stderr, "%s: %s (%s)\n", what, fk_status_string(s), fk_last_error());
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: %s FRAME W H OUT_W OUT_H STRICT CROPS OUT\n", argv[0]);
        return 1;
    }
    const int W = atoi(argv[2]), H = atoi(argv[3]), OW = atoi(argv[4]), OH = atoi(argv[5]);
    const int strict = atoi(argv[6]);
    if (W < 1 || H < 1 || OW < 1 || OH < 1)
        return 1;

    static int crop[MAX_CROPS][4];
    int n = 0;
    FILE *fc = fopen(argv[7], "r");
    if (!fc)
        return 1;
    while (n < MAX_CROPS && fscanf(fc, "%d %d %d %d", &crop[n][0], &crop[n][1], &crop[n][2], &crop[n][3]) == 4)
        ++n;
    fclose(fc);
    if (n == 0)
        return 1;

    const size_t frame_bytes = (size_t)W * H * 3;
    unsigned char *h_frame = (unsigned char *)malloc(frame_bytes);
    FILE *ff = fopen(argv[1], "rb");
    if (!h_frame || !ff || fread(h_frame, 1, frame_bytes, ff) != frame_bytes)
        return 1;
    fclose(ff);

    /* the chain: constants in fp32, per channel after the swap (RGB order) */
    const float scale = 1.0f / 255.0f;
    const float mean[3] = {0.485f, 0.456f, 0.406f};
    const float stdv[3] = {0.229f, 0.224f, 0.225f};
    printf("scale %a\nmean %a %a %a\nstd %a %a %a\n", scale, mean[0], mean[1], mean[2], stdv[0],
           stdv[1], stdv[2]);
    fk_op_desc ops[5] = {
        {FK_OP_SWAP_RB, 0, {0, 0, 0, 0}, 0, 0},
        {FK_OP_CVT_F32, 0, {0, 0, 0, 0}, 0, 0},
        {FK_OP_MUL, 1, {scale, 0, 0, 0}, 0, 0},
        {FK_OP_SUB, 3, {mean[0], mean[1], mean[2], 0}, 0, 0},
        {FK_OP_DIV, 3, {stdv[0], stdv[1], stdv[2], 0}, 0, 0},
    };
    fk_chain_desc chain;
    chain.read.kind = FK_READ_CROP_RESIZE;
    chain.read.in_dtype = FK_U8;
    chain.read.channels = 3;
    chain.ops = ops;
    chain.n_ops = 5;
    chain.write.out_dtype = FK_F32;
    chain.write.layout = FK_PLANAR;

    fk_plan_opts opts = {FK_CONFIG_DEFAULT, {256, 1}, 0, strict, FK_TIER_AUTO, 0, FK_GATHER_DIRECT};

    const size_t out_elems = (size_t)3 * OW * OH;
    const size_t out_bytes = sizeof(float) * out_elems * (size_t)n;
    void *d_frame = NULL, *d_out = NULL;
    hipStream_t stream = NULL;
    fk_plan *plan = NULL;
    int rc = 2;
    float *h_out = (float *)malloc(out_bytes);
    fk_item *items = (fk_item *)calloc((size_t)n, sizeof(fk_item));
    if (!h_out || !items)
        return 1;
    if (!hip_ok(hipMalloc(&d_frame, frame_bytes), "hipMalloc frame") ||
        !hip_ok(hipMalloc(&d_out, out_bytes), "hipMalloc out") ||
        !hip_ok(hipStreamCreate(&stream), "hipStreamCreate") ||
        !hip_ok(hipMemcpy(d_frame, h_frame, frame_bytes, hipMemcpyHostToDevice), "hipMemcpy frame"))
        goto done;
    for (int i = 0; i < n; ++i) {
        items[i].src.ptr = d_frame;
        items[i].src.width = W;
        items[i].src.height = H;
        items[i].src.pitch_bytes = (int64_t)W * 3;
        items[i].x = crop[i][0];
        items[i].y = crop[i][1];
        items[i].w = crop[i][2];
        items[i].h = crop[i][3];
        items[i].dst = (float *)d_out + out_elems * (size_t)i;
        items[i].out_w = OW;
        items[i].out_h = OH;
    }
    if (!fk_ok(fk_plan_create(&chain, n, &opts, &plan), "fk_plan_create") ||
        !fk_ok(fk_run(plan, items, n, (void *)stream), "fk_run") ||
        !hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize") ||
        !hip_ok(hipMemcpy(h_out, d_out, out_bytes, hipMemcpyDeviceToHost), "hipMemcpy out"))
        goto done;
    FILE *fo = fopen(argv[8], "wb");
    if (!fo || fwrite(h_out, 1, out_bytes, fo) != out_bytes) {
        rc = 1;
        goto done;
    }
    fclose(fo);
    printf("ran %d crops with %s\n", n, fk_version());
    rc = 0;
done:
    if (plan)
        fk_plan_destroy(plan);
    if (stream)
        (void)hipStreamDestroy(stream);
    if (d_out)
        (void)hipFree(d_out);
    if (d_frame)
        (void)hipFree(d_frame);
    free(items);
    free(h_out);
    free(h_frame);
    return rc;
}

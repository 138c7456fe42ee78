"""The oracle's pins are strong enough: each plausible mistake planted in a
copy of the oracle (a dropped term, a wrong sign or index, a transposed
operand) makes at least one pin fail.  Runs on the CPU only."""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
import test_oracle_f64_pins as dpins
import test_oracle_pins as pins
import test_oracle_read_pins as rpins
import test_oracle_stats_pins as spins

SRC = open(oracle.SRC).read()

# (name, text in fk_oracle.c, planted replacement); every variant stays in
# bounds of its buffers
MUTATIONS = [
    ("half-pixel offset dropped", "fmaf((float)o + 0.5f, scale, -0.5f)", "fmaf((float)o + 0.5f, scale, 0.0f)"),
    ("vertical lerp uses the x weight", "float v = fmaf(ay, bot - top, top);", "float v = fmaf(ax, bot - top, top);"),
    ("second tap dropped", "*i1 = lo + 1 < in_size ? lo + 1 : in_size - 1;", "*i1 = lo;"),
    ("coordinate not clamped at 0", "    if (s < 0.0f)\n        s = 0.0f;\n", ""),
    ("swap exchanges channels 0 and 1", "size_t a = p * (size_t)m->C, b = a + 2;", "size_t a = p * (size_t)m->C, b = a + 1;"),
    ("per-channel constant index ignored", "float k = op->nconst == 1 ? op->k[0] : op->k[c];", "float k = op->k[0];"),
    ("planar plane transposed",
     "((size_t)c * (size_t)m->h + (size_t)y) * (size_t)m->w + (size_t)x",
     "((size_t)c * (size_t)m->w + (size_t)x) * (size_t)m->h + (size_t)y"),
    ("subtraction sign flipped", "case ORC_SUB: r = v - k;", "case ORC_SUB: r = k - v;"),
    ("division by reciprocal", "default:      r = v / k;", "default:      r = v * (1.0f / k);"),
    ("crop x offset dropped", "frame_elem(it, ch->in_dtype, C, it->x + i, it->y + j, c)", "frame_elem(it, ch->in_dtype, C, i, it->y + j, c)"),
    ("fp16 rounding truncates", "double q = nearbyint(ldexp(a, -ulp_exp));", "double q = floor(ldexp(a, -ulp_exp));"),
    ("mul and add exchanged", "case ORC_MUL: r = v * k;", "case ORC_MUL: r = v + k;"),
    ("loop runs its body once too often", "for (int32_t r = 1; r < op->count; ++r)",
     "for (int32_t r = 0; r < op->count; ++r)"),
    ("nearest drops the half-pixel centre", "int64_t sx = ((int64_t)2 * ox + 1) * in->w",
     "int64_t sx = ((int64_t)2 * ox) * in->w"),
    ("NV12 chroma row from y/4", "((int64_t)it->H + y / 2) * it->pitch", "((int64_t)it->H + y / 4) * it->pitch"),
    ("NV12 green takes +v", "out[1] = (c - 0.813f * v) - 0.391f * u;", "out[1] = (c + 0.813f * v) - 0.391f * u;"),
    ("NV12 U and V exchanged", "float u = (float)uv[0] - 128.0f;", "float u = (float)uv[1] - 128.0f;"),
    ("stats min takes the maximum", "mn = fminf(mn, v);", "mn = fmaxf(mn, v);"),
    ("stats read channel 0 only", "float v = m->v[p * (size_t)C + (size_t)c];", "float v = m->v[p * (size_t)C];"),
    ("stats mean over one row", "out[4 * c + 3] = sum / (double)npix;", "out[4 * c + 3] = sum / (double)m->w;"),
    ("fp64 write stores the fp32 chain", "((double *)it->dst)[o] = m->d[i];",
     "((double *)it->dst)[o] = (double)m->v[i];"),
    ("fp64 frame read through fp32", "out->d[o] = d;", "out->d[o] = (double)(float)d;"),
    ("fp64 multiply rounded to fp32", "case ORC_MUL: r = v * k; rd = d * (double)k;",
     "case ORC_MUL: r = v * k; rd = (double)(float)(d * (double)k);"),
    ("loop skips the first op of its body",
     "for (int32_t j = i - op->span; j < i; ++j)\n                        step_arith",
     "for (int32_t j = i - op->span + 1; j < i; ++j)\n                        step_arith"),
]

PINS = [
    ("test_resize_same_size_is_identity", {}),
    ("test_resize_constant_image_stays_constant", {"src": (100, 60), "dst": (37, 91)}),
    ("test_resize_linear_ramp_is_source_coordinate", {"w": 200, "h": 150, "ow": 64, "oh": 128}),
    ("test_resize_linear_ramp_is_source_coordinate", {"w": 60, "h": 90, "ow": 224, "oh": 224}),
    ("test_resize_integer_downscale_is_box_mean", {"f": 2}),
    ("test_resize_2x_upscale_weights_quarter_three_quarters", {}),
    ("test_resize_matches_torch_bilinear", {"seed": 0}),
    ("test_crop_swap_split_index_coded", {"layout": "planar", "kind": "crop_resize"}),
    ("test_crop_swap_split_index_coded", {"layout": "packed", "kind": "plain"}),
    ("test_per_channel_constants_follow_swapped_positions", {}),
    ("test_normalise_chain_is_per_op_ieee_fp32", {}),
    ("test_muladd_chain_matches_affine_closed_form", {"n_ops": 4}),
    ("test_loop_equals_unrolled_body", {"span": 3, "count": 4}),
    ("test_loop_chain_matches_affine_closed_form", {"pairs": 7}),
    ("test_stats_of_coordinate_ramps_are_closed_forms", {"roi": (3, 5, 17, 9)}),
    ("test_nearest_integer_downscale_takes_centre_pixel", {"f": 3}),
    ("test_nv12_bt601_colour_table", {"yuv": (81, 90, 240), "rgb": (255, 0, 0)}),
    ("test_nv12_bt601_colour_table", {"yuv": (145, 54, 34), "rgb": (0, 255, 0)}),
    ("test_nv12_chroma_pair_serves_a_2x2_block", {}),
    ("test_division_is_true_division_not_reciprocal", {}),
    ("test_float_to_half_round_to_nearest_even_matches_numpy", {}),
    ("test_each_op_rounds_once_to_double", {"in_dtype": "f64"}),
]


def build_variant(src_text, path, extra=()):
    c = path + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
                           *extra, "-shared", "-w", "-o", path, c, "-lm"])


def load_as_oracle(path, monkeypatch):
    L = ctypes.CDLL(path)
    real = oracle.lib()
    for name in ("orc_run", "orc_validate", "orc_resize_f32", "orc_half_to_float", "orc_float_to_half"):
        fn = getattr(L, name)
        fn.argtypes = getattr(real, name).argtypes
        fn.restype = getattr(real, name).restype
    monkeypatch.setattr(oracle, "_lib", L)


def caught_by_pins():
    for name, kw in PINS:
        try:
            (getattr(pins, name, None) or getattr(spins, name, None) or getattr(dpins, name, None) or
             getattr(rpins, name))(**kw)
        except AssertionError:
            return name
    return None


def test_unmodified_oracle_passes_the_pin_subset(monkeypatch):
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "orig.so")
        build_variant(SRC, path)
        load_as_oracle(path, monkeypatch)
        assert caught_by_pins() is None


def test_oracle_has_no_undefined_behaviour_on_the_pins(monkeypatch):
    """The oracle built with the undefined-behaviour sanitizer (integer
    overflow, shifts, out-of-bounds indexing of fixed arrays, misaligned
    access; any report aborts) runs the pin subset and passes it."""
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ubsan.so")
        build_variant(SRC, path, ("-fsanitize=undefined", "-fno-sanitize-recover=undefined"))
        load_as_oracle(path, monkeypatch)
        assert caught_by_pins() is None


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, monkeypatch):
    assert SRC.count(old) == 1, f"mutation site for '{name}' not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mut.so")
        build_variant(SRC.replace(old, new), path)
        load_as_oracle(path, monkeypatch)
        assert caught_by_pins() is not None, f"no pin caught: {name}"

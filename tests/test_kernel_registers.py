"""Register use of the built kernels (CPU only): no fused transform or stats
kernel may spill to scratch, since spilled tiles made launches 4-5x slower.
Reads the code objects' metadata notes out of libfkmi.so with the ROCm
LLVM tools; skipped when the library or the tools are missing."""
import os
import re
import subprocess
import tempfile

import pytest

import paper_2508_07071_amd as fk

LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"

# kernels allowed a few dwords of scratch: the run-time op list into packed
# output at K = 8 (and the NV12 read at K = 4), at most 16 bytes each
OPLIST_PACKED = re.compile(r"^_ZN2fk11k_transformI.*RuntimeComputeENS_11WritePackedILi\dELi3EEELi3ELi[48]E")


def kernel_metadata():
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not os.path.exists(fk.LIB_PATH) or not all(os.path.exists(t) for t in tools):
        pytest.skip("libfkmi.so or the ROCm LLVM tools are missing")
    objcopy, bundler, readelf = tools
    out = {}
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fatbin")
        subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", fk.LIB_PATH, os.path.join(d, "lib")],
                       check=True, capture_output=True)
        blob = open(fat, "rb").read()
        starts = [m.start() for m in re.finditer(re.escape(MAGIC), blob)]
        assert starts, "no offload bundles in libfkmi.so"
        for i, s in enumerate(starts):
            part = os.path.join(d, f"b{i}")
            dev = os.path.join(d, f"d{i}.o")
            end = starts[i + 1] if i + 1 < len(starts) else len(blob)
            open(part, "wb").write(blob[s:end])
            subprocess.run([bundler, "--type=o", f"--input={part}", f"--targets={TARGET}", f"--output={dev}",
                            "--unbundle"], check=True, capture_output=True)
            notes = subprocess.run([readelf, "--notes", dev], check=True, capture_output=True, text=True).stdout
            name = None
            for line in notes.splitlines():
                m = re.match(r"\s+\.name:\s+(\S+)", line)
                if m:
                    name = m.group(1)
                    out[name] = {}
                    continue
                m = re.match(r"\s+\.(private_segment_fixed_size|vgpr_count|vgpr_spill_count):\s+(\d+)", line)
                if m and name:
                    out[name][m.group(1)] = int(m.group(2))
    return out


def test_no_fused_kernel_spills_its_tile():
    meta = kernel_metadata()
    assert len(meta) > 500, f"only {len(meta)} kernels found"
    bad = []
    for name, m in meta.items():
        scratch = m.get("private_segment_fixed_size", 0)
        if scratch == 0:
            continue
        if OPLIST_PACKED.match(name) and scratch <= 16:
            continue
        bad.append((name, scratch))
    assert not bad, f"{len(bad)} kernels use scratch: {bad[:5]}"


def test_depth_sweep_kernels_stay_in_registers():
    """The benchmark's compile-time chains at every coarsening, the
    crop+resize normalise kernels, the u8 stats kernels and the fp64 chains
    use no scratch."""
    meta = kernel_metadata()
    hot = [n for n in meta if "OpMulAddLoop" in n or "k_resize_px" in n or "k_stats_u8" in n or "k_f64" in n]
    assert len(hot) >= 16
    for n in hot:
        assert meta[n].get("private_segment_fixed_size", 0) == 0, n

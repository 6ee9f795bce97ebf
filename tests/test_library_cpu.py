"""CPU-side checks of the HIP library: it loads, exports every symbol that
include/rips.h declares, and rejects bad arguments before any HIP call."""

import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rips.h")


def _header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rips_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1908_02518_amd as rips
    out = subprocess.run(["nm", "-D", "--defined-only", rips.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rips_\w+)", out))
    declared = _header_functions()
    assert declared, "no declarations found"
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        getattr(rips.lib(), f)


def test_binding_lists_the_header():
    import paper_1908_02518_amd as rips
    assert sorted(rips.EXPORTS) == _header_functions()


def test_status_strings():
    import paper_1908_02518_amd as rips
    for code in rips.STATUS:
        assert rips.lib().rips_status_string(code)


@pytest.mark.parametrize("kw,code", [
    (dict(p=4), -2),
    (dict(p=1), -2),
    (dict(p=65537), -2),
    (dict(max_dim=4), -1),
    (dict(max_dim=-1), -1),
    (dict(threshold=float("nan")), -1),
])
def test_argument_validation_before_any_hip_call(kw, code):
    import paper_1908_02518_amd as rips
    x = np.zeros((5, 2), np.float32)
    args = dict(max_dim=1, threshold=float("inf"), p=2)
    args.update(kw)
    with pytest.raises(rips.RipsError) as e:
        rips.barcode(x, **args)
    assert e.value.status == code


def test_index_overflow_rejected():
    import paper_1908_02518_amd as rips
    # C(65535, 5) > 2^63
    n = 65535
    assert math.comb(n, 5) >= 2 ** 63
    lib = rips.lib()
    out = ctypes.POINTER(rips.rips_result)()
    dummy = (ctypes.c_float * 1)()
    st = lib.rips_barcode(dummy, n, 1, 3, ctypes.c_float(1.0), 2, ctypes.byref(out))
    assert st == -3 and not out


def test_empty_and_null_inputs_rejected():
    import paper_1908_02518_amd as rips
    lib = rips.lib()
    out = ctypes.POINTER(rips.rips_result)()
    assert lib.rips_barcode(None, 4, 2, 1, ctypes.c_float(1.0), 2, ctypes.byref(out)) == -1
    dummy = (ctypes.c_float * 1)()
    assert lib.rips_barcode(dummy, 0, 2, 1, ctypes.c_float(1.0), 2, ctypes.byref(out)) == -1
    assert lib.rips_barcode(dummy, 4, -1, 1, ctypes.c_float(1.0), 2, ctypes.byref(out)) == -1


def test_backward_validation_before_any_hip_call():
    import paper_1908_02518_amd as rips
    lib = rips.lib()
    d = ctypes.c_void_p(8)  # never dereferenced: rejected before any HIP call
    # n out of range, k_birth out of range, distance input with row offsets,
    # negative bar count
    assert lib.rips_backward_device(d, 0, 2, 1, 1, None, d, d, d, d, d, None) == -1
    assert lib.rips_backward_device(d, 10, 2, 1, 9, None, d, d, d, d, d, None) == -1
    assert lib.rips_backward_device(d, 10, 0, 1, 1, d, d, d, d, d, d, None) == -1
    assert lib.rips_backward_device(d, 10, 2, -1, 1, None, d, d, d, d, d, None) == -1
    # nothing to do
    assert lib.rips_backward_device(d, 10, 2, 0, 1, None, d, d, d, d, d, None) == 0


def test_batched_config_validation():
    import paper_1908_02518_amd as rips
    lib = rips.lib()
    # rejected before the device context is touched
    assert lib.rips_batched_set_config(3000, 1) == -1
    assert lib.rips_batched_set_config(1024, 9) == -1
    assert lib.rips_set_reduce_workgroups(-1) == -1
    assert lib.rips_set_shortcuts(-1) == -1
    assert lib.rips_set_shortcuts(8) == -1
    assert lib.rips_set_reduced_storage(4) == -1
    assert lib.rips_set_reduced_storage(-1) == -1
    assert lib.rips_batched_autotune(None, None, 1, 2, 8, 1, ctypes.c_float(1.0), 2, None, None,
                                     0, None, None, None) == -1


def _record_layouts(src: str, side: str):
    """{record: (size, field offsets)} of the rips:: records as one compiler
    pass (host or device) lays them out."""
    csrc = os.path.join(ROOT, "paper_1908_02518_amd", "csrc")
    r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++17", "-I",
                        os.path.join(ROOT, "include"), f"--cuda-{side}-only", "-fsyntax-only", src,
                        "-Xclang", "-fdump-record-layouts-simple"],
                       capture_output=True, text=True, cwd=csrc)
    out = {}
    for blk in r.stdout.split("*** Dumping AST Record Layout")[1:]:
        t = re.search(r"Type: (.*)", blk).group(1).strip()
        if "rips::" in t:
            out[t] = (re.search(r"Size:(\d+)", blk).group(1),
                      re.search(r"FieldOffsets: \[(.*?)\]", blk).group(1))
    return out


def _kernel_argument_records(src: str):
    """Record names that appear in the parameter lists of the file's kernels."""
    text = open(os.path.join(ROOT, "paper_1908_02518_amd", "csrc", src)).read()
    text = re.sub(r"__launch_bounds__\s*\([^)]*\)", "", text)
    names = set()
    for m in re.finditer(r"__global__[^{;]*?\w+\s*\(([^)]*)\)", text, flags=re.S):
        names.update(re.findall(r"\b([A-Z]\w*)\b", m.group(1)))
    return names


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
@pytest.mark.parametrize("src", ["rips_kernels.hip", "rips_batched.hip"])
def test_kernel_argument_layouts_match_between_host_and_device(src):
    # a record passed by value to a kernel is laid out by the host and read by
    # the device: an LDS pointer (32 bits on the device, 64 on the host) in
    # one would shift every later field
    host, dev = _record_layouts(src, "host"), _record_layouts(src, "device")
    wanted = _kernel_argument_records(src)
    assert wanted
    checked = 0
    for t, lay in host.items():
        short = re.sub(r"^struct |^class ", "", t).replace("rips::", "").split("<")[0]
        if short in wanted:
            assert dev.get(t) == lay, (t, lay, dev.get(t))
            checked += 1
    assert checked >= 2


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _misplaced_copies(asm: str):
    """Register copies of the allocator (moves to or from the accumulation
    registers, spill stores and reloads) placed at the end of a divergent
    region, just before its exec mask is restored: they run only in the
    region's lanes, and a value the other lanes need afterwards is then
    undefined in them."""
    lines = asm.splitlines()
    kinds = ("v_accvgpr_write_b32", "v_accvgpr_read_b32", "scratch_store", "scratch_load")
    hits = []
    for i, ln in enumerate(lines):
        if not re.match(r"\s*s_or_b64 exec, exec, s\[\d+:\d+\]\s*$", ln):
            continue
        j = i - 1
        while j >= 0:
            t = lines[j].strip()
            if lines[j].startswith((".LBB", "; %bb")) or t.endswith(":"):
                break
            if t.startswith(kinds) and "Folded" not in t:
                hits.append((i + 1, t))
            elif t and not t.startswith((";", "s_waitcnt", "s_nop")):
                break
            j -= 1
    return hits


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
@pytest.mark.parametrize("src", ["rips_batched.hip", "rips_kernels.hip"])
def test_no_register_copy_before_exec_restore(src, tmp_path):
    # a compiler placement once put a copy of max_dim into an accumulation
    # register at the end of a divergent loop; the lanes outside the loop then
    # read an undefined max_dim and took the dimension-1 branch alone
    csrc = os.path.join(ROOT, "paper_1908_02518_amd", "csrc")
    out = str(tmp_path / "k.s")
    r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                        "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
                        "--cuda-device-only", "-S", src, "-o", out],
                       capture_output=True, text=True, cwd=csrc, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    hits = _misplaced_copies(open(out).read())
    assert not hits, hits[:5]


def test_misplaced_copy_scanner_finds_the_pattern():
    # the shape the scanner looks for, as the compiler once emitted it, and a
    # correct join block (the copy after the exec restore)
    bad = "\n".join([".LBB8_104:", "\tv_accvgpr_write_b32 a4, v24",
                     "\ts_or_b64 exec, exec, s[0:1]", "\ts_getpc_b64 s[2:3]"])
    good = "\n".join([".LBB8_104:", "\ts_or_b64 exec, exec, s[0:1]",
                      "\tv_accvgpr_write_b32 a4, v24", "\ts_getpc_b64 s[2:3]"])
    assert _misplaced_copies(bad) == [(3, "v_accvgpr_write_b32 a4, v24")]
    assert _misplaced_copies(good) == []

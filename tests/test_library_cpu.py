"""Host-side checks of the C-ABI library that need no GPU: the library loads,
exports every entry point the header declares, its struct layouts match the
header as compiled by a C compiler, and argument errors are reported without
touching the device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from conftest import ROOT
from paper_2212_01473_amd import mce

HEADER = os.path.join(ROOT, "include", "mce.h")


def test_library_loads_and_exports_header_symbols():
    lib = mce.load_library()
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:mce_status|void|const char\*)\s+(mce_\w+)\s*\(", text, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(mce.EXPORTED)
    out = subprocess.check_output(["nm", "-D", "--defined-only", mce.LIB_PATH]).decode()
    exported = set(re.findall(r" T (mce_\w+)", out))
    assert declared <= exported
    for name in declared:
        assert hasattr(lib, name)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    m = re.search(r"#define MCE_NOALLOC_MAX_SAMPLES (\d+)u", text)
    assert m and int(m.group(1)) == mce.MCE_NOALLOC_MAX_SAMPLES
    m = re.search(r"#define MCE_MODEL_FLOATS (\d+)", text)
    assert m and int(m.group(1)) == mce.MODEL_FLOATS
    m = re.search(r"#define MCE_GRAPH_WHOLE (0x[0-9A-Fa-f]+)u", text)
    assert m and int(m.group(1), 16) == mce.GRAPH_WHOLE


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "mce.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("mce_options %zu\n", sizeof(mce_options));
  printf("mce_result %zu\n", sizeof(mce_result));
  printf("mce_graph_info %zu\n", sizeof(mce_graph_info));
  printf("mce_tune_report %zu\n", sizeof(mce_tune_report));
  F(mce_options, model); F(mce_options, stream); F(mce_options, timeout_ms); F(mce_options, root_nodes);
  F(mce_options, xrow_min_u); F(mce_options, xrow_budget_words); F(mce_options, task_log);
  F(mce_options, task_log_cap);
  F(mce_result, hist); F(mce_result, stream_vertices); F(mce_result, stats);
  F(mce_graph_info, n_isolated); F(mce_graph_info, n_graphs);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().splitlines())
    got = {k: int(v) for k, v in got.items()}
    assert got["mce_options"] == C.sizeof(mce.Options)
    assert got["mce_result"] == C.sizeof(mce.Result)
    assert got["mce_graph_info"] == C.sizeof(mce.GraphInfo)
    assert got["mce_tune_report"] == C.sizeof(mce.TuneReport)
    assert got["mce_options.model"] == mce.Options.model.offset
    assert got["mce_options.stream"] == mce.Options.stream.offset
    assert got["mce_options.timeout_ms"] == mce.Options.timeout_ms.offset
    assert got["mce_options.root_nodes"] == mce.Options.root_nodes.offset
    assert got["mce_options.xrow_min_u"] == mce.Options.xrow_min_u.offset
    assert got["mce_options.xrow_budget_words"] == mce.Options.xrow_budget_words.offset
    assert got["mce_options.task_log"] == mce.Options.task_log.offset
    assert got["mce_options.task_log_cap"] == mce.Options.task_log_cap.offset
    assert got["mce_result.hist"] == mce.Result.hist.offset
    assert got["mce_result.stream_vertices"] == mce.Result.stream_vertices.offset
    assert got["mce_result.stats"] == mce.Result.stats.offset
    assert got["mce_graph_info.n_isolated"] == mce.GraphInfo.n_isolated.offset
    assert got["mce_graph_info.n_graphs"] == mce.GraphInfo.n_graphs.offset


def test_status_strings_and_version():
    lib = mce.load_library()
    for code in range(-7, 2):
        s = lib.mce_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.mce_status_string(-100).decode() == "unknown status"
    assert "gfx950" in mce.version()


def test_argument_errors_without_device():
    lib = mce.load_library()
    h = C.c_void_p()
    # NULL out pointer
    assert lib.mce_load_csr(None, None, 0, 0, 0, None, None) == mce.MCE_ERR_INVALID_ARG
    # NULL row_ptr
    assert lib.mce_load_csr(None, None, 0, 0, 0, None, C.byref(h)) == mce.MCE_ERR_INVALID_ARG
    assert "row_ptr" in lib.mce_last_error().decode()
    # unknown load flag
    rp = (C.c_uint32 * 1)(0)
    assert lib.mce_load_csr(C.cast(rp, C.c_void_p), None, 0, 0, 0x100, None, C.byref(h)) == mce.MCE_ERR_INVALID_ARG
    # enumerate / info on NULL handles
    r = mce.Result()
    assert lib.mce_enumerate(None, None, C.byref(r)) == mce.MCE_ERR_INVALID_ARG
    gi = mce.GraphInfo()
    assert lib.mce_graph_get_info(None, 0, C.byref(gi)) == mce.MCE_ERR_INVALID_ARG
    assert lib.mce_graph_copy_order(None, 0, None, None, None) == mce.MCE_ERR_INVALID_ARG
    assert lib.mce_enumerate_batch(None, None, C.byref(r), 1) == mce.MCE_ERR_INVALID_ARG
    o = mce.Options()
    assert lib.mce_autotune(None, C.byref(o), C.byref(o), None) == mce.MCE_ERR_INVALID_ARG
    lib.mce_free(None)


def test_binding_fails_loudly_without_library(tmp_path):
    saved = mce._lib
    mce._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            mce.load_library(str(tmp_path / "missing.so"))
    finally:
        mce._lib = saved


def test_options_carry_learned_flags():
    import torch

    model = torch.zeros(mce.MODEL_FLOATS)
    o = mce.make_options(model=model, split=True)
    assert o.flags & mce.F_LEARNED_ORDER and o.flags & mce.F_SPLIT and o.flags & mce.F_WORKER_LIST
    assert o.model == model.data_ptr()
    o = mce.make_options(model=model)
    assert o.flags & mce.F_LEARNED_ORDER and not o.flags & mce.F_SPLIT
    o = mce.make_options()
    assert not o.flags & (mce.F_LEARNED_ORDER | mce.F_SPLIT)
    with pytest.raises(ValueError):
        mce.make_options(split=True)


def test_stat_names_cover_header_indices():
    # one binding name per MCE_STAT_* index, in index order, within stats[]
    text = open(HEADER).read()
    idx = sorted(int(v) for v in re.findall(r"MCE_STAT_\w+\s*=\s*(\d+)", text))
    assert idx == list(range(len(idx)))
    assert len(mce.STAT_NAMES) == len(idx)
    size = int(re.search(r"uint64_t stats\[(\d+)\]", text).group(1))
    assert len(idx) <= size


def test_enumeration_kernel_resources():
    """The build records each kernel's resources from the compiler; the DFS
    kernel's two instantiations must keep 5 and 6 wavefronts per SIMD (a
    silent register-allocation change costs resident workgroups), paid for
    with at most 40 and 56 spilled words per lane."""
    import json

    from paper_2212_01473_amd import build

    if not os.path.exists(build.RESOURCES):
        pytest.skip("library not built in this tree")
    res = json.load(open(build.RESOURCES))
    k = {name: v for name, v in res.items() if "k_enumerate" in name}
    assert len(k) == 2, list(k)
    five = [v for name, v in k.items() if "ILi5E" in name]
    six = [v for name, v in k.items() if "ILi6E" in name]
    assert len(five) == 1 and len(six) == 1, list(k)
    assert five[0]["occupancy"] >= 5 and five[0]["vgprs"] <= 96 and five[0]["scratchsize"] <= 160, five[0]
    assert six[0]["occupancy"] >= 6 and six[0]["vgprs"] <= 80 and six[0]["scratchsize"] <= 224, six[0]
    for kernel in ("k_mlp_infer_bf16", "k_features", "k_pd_decrement", "scan"):
        for name, v in res.items():
            if kernel in name:
                assert v["scratchsize"] == 0, name


def test_enumeration_kernel_makes_no_calls(tmp_path):
    """The enumeration kernel's helpers read the kernel parameters through the
    kernel-argument pointer, which only the kernel itself has: an outlined
    (called) helper would read them from address zero.  Every such helper is
    force-inlined; the device assembly must contain no call."""
    import shutil
    import subprocess

    from paper_2212_01473_amd import build

    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    src = os.path.join(build.CSRC, "enumerate.hip")
    out = tmp_path / "enumerate.s"
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC", "-Rpass-analysis=kernel-resource-usage")]
    flags += build.SOURCE_FLAGS.get("enumerate.hip", [])
    subprocess.run([build.HIPCC, *flags, "--cuda-device-only", "-S", src, "-o", str(out)], check=True,
                   capture_output=True, timeout=600)
    text = out.read_text()
    assert "s_swappc_b64" not in text and "s_setpc_b64" not in text
    shutil.rmtree(tmp_path, ignore_errors=True)


def test_search_asm_registers_are_declared():
    """The folded executor's assembly search loop may only touch registers its
    asm statement names: operands (pinned with explicit register constraints)
    or clobbers.  An undeclared register would silently corrupt a value the
    compiler keeps there."""
    from paper_2212_01473_amd import build

    src = open(os.path.join(build.CSRC, "enumerate.hip")).read()
    body = src[src.index("#define FOLDED_SEARCH_ASM"):]
    body = body[:body.index('"s_nop 4\\n"', body.index(".Lfs_exit_")) + 12]
    code = "".join(re.findall(r'"([^"]*)\\n"', body))

    def expand(tok):
        m = re.fullmatch(r"([sv])\[(\d+):(\d+)\]", tok)
        if m:
            return {f"{m.group(1)}{i}" for i in range(int(m.group(2)), int(m.group(3)) + 1)}
        return {tok}

    used = set()
    for tok in re.findall(r"\b[sv]\[\d+:\d+\]|\b[sv]\d+\b", code):
        used |= expand(tok)
    stmt = src[src.index("asm volatile(FOLDED_SEARCH_ASM"):]
    stmt = stmt[:stmt.index(");")]
    declared = set()
    for tok in re.findall(r'"\+?\{([sv]\[\d+:\d+\]|[sv]\d+)\}"', stmt):
        declared |= expand(tok)
    for tok in re.findall(r'"([sv]\d+)"', stmt):
        declared |= expand(tok)
    assert used, "no registers parsed from the assembly"
    assert used <= declared, sorted(used - declared)
    # m0 is saved and restored by the block itself, never declared
    assert "s_mov_b32 s76, m0" in code and "s_mov_b32 m0, s76" in code
    assert "s76" in declared

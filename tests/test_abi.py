"""The C ABI library without a GPU: it loads, exports every symbol the
header declares, its structs match the Python binding, and argument errors
come back as the documented codes before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1508_06329_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lexbfs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|int32_t|size_t|char|void)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblexbfs.so not built")
    return _lib.load()


def test_header_declares_the_binding_list():
    assert declared_functions() == sorted(_lib.EXPORTED)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(rf"\bT {name}$", out, flags=re.M), name


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lexbfs.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lexbfs_graph_t), '
                   'offsetof(lexbfs_graph_t, nnz), offsetof(lexbfs_graph_t, bits), offsetof(lexbfs_graph_t, words_per_row), '
                   'sizeof(lexbfs_result_t), sizeof(lexbfs_outputs_t), sizeof(lexbfs_tuning_t)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    exp = [ctypes.sizeof(_lib.lexbfs_graph_t), _lib.lexbfs_graph_t.nnz.offset, _lib.lexbfs_graph_t.bits.offset,
           _lib.lexbfs_graph_t.words_per_row.offset, ctypes.sizeof(_lib.lexbfs_result_t),
           ctypes.sizeof(_lib.lexbfs_outputs_t), ctypes.sizeof(_lib.lexbfs_tuning_t)]
    assert got == exp
    assert got[4] == 32


def fake_graph(n, W=None, nnz=10):
    g = _lib.lexbfs_graph_t()
    g.n = n
    g.reserved = 0
    g.nnz = nnz
    # non-null placeholders: argument checks never dereference them
    g.row_ptr = 0x1000
    g.col_idx = 0x2000
    g.bits = 0x3000
    g.words_per_row = (n + 63) // 64 if W is None else W
    return g


def test_argument_errors(lib):
    ws_need = lib.lexbfs_workspace_bytes(100)
    ws = 0x10000
    res = 0x20000
    order = 0x30000
    assert lib.lexbfs_order(None, order, None, None, ws, ws_need, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(-1)
    assert lib.lexbfs_order(ctypes.byref(g), order, None, None, ws, ws_need, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(_lib.LEXBFS_MAX_N + 1)
    assert lib.lexbfs_order(ctypes.byref(g), order, None, None, ws, 1 << 40, None) == _lib.LEXBFS_ETOOBIG
    g = fake_graph(100, W=1)
    assert lib.lexbfs_order(ctypes.byref(g), order, None, None, ws, ws_need, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(100)
    assert lib.lexbfs_order(ctypes.byref(g), order, None, None, ws, ws_need - 1, None) == _lib.LEXBFS_ENOWS
    assert lib.lexbfs_order(ctypes.byref(g), order, None, None, None, ws_need, None) == _lib.LEXBFS_ENOWS
    assert lib.lexbfs_order(ctypes.byref(g), None, None, None, ws, ws_need, None) == _lib.LEXBFS_EINVAL
    g.reserved = 1
    assert lib.chordal_test(ctypes.byref(g), res, None, ws, ws_need, 0, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(100)
    g.nnz = 1 << 31
    assert lib.chordal_test(ctypes.byref(g), res, None, ws, ws_need, 0, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(100)
    g.bits = None
    assert lib.chordal_test(ctypes.byref(g), res, None, ws, ws_need, 0, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(100)
    assert lib.chordal_test(ctypes.byref(g), None, None, ws, ws_need, 0, None) == _lib.LEXBFS_EINVAL
    assert lib.chordal_test(ctypes.byref(g), res, None, ws, 16, 0, None) == _lib.LEXBFS_ENOWS
    # batch
    arr = (_lib.lexbfs_graph_t * 2)(fake_graph(10), fake_graph(-3))
    assert lib.chordal_test_batch(arr, 2, None, res, None, ws, 1 << 30, 0, None) == _lib.LEXBFS_EINVAL
    assert lib.chordal_test_batch(arr, -1, None, res, None, ws, 1 << 30, 0, None) == _lib.LEXBFS_EINVAL
    assert lib.chordal_test_batch(arr, 0, None, res, None, ws, 0, 0, None) == _lib.LEXBFS_OK
    arr = (_lib.lexbfs_graph_t * 2)(fake_graph(10), fake_graph(70000))
    assert lib.chordal_test_batch(arr, 2, None, res, None, ws, 1 << 30, 0, None) == _lib.LEXBFS_ETOOBIG
    tun = _lib.lexbfs_tuning_t(0, 999, 0, 0)
    arr = (_lib.lexbfs_graph_t * 1)(fake_graph(10))
    assert lib.chordal_test_batch(arr, 1, None, res, ctypes.byref(tun), ws, 1 << 30, 0, None) == _lib.LEXBFS_EINVAL
    small = lib.lexbfs_batch_workspace_bytes(arr, 1)
    assert lib.chordal_test_batch(arr, 1, None, res, None, ws, 0, 0, None) == _lib.LEXBFS_ENOWS
    assert small > 0
    plan = ctypes.c_void_p()
    assert lib.lexbfs_batch_plan_create(arr, 1, None, res, None, ws, 0, 0, None, None) == _lib.LEXBFS_EINVAL
    assert lib.lexbfs_batch_plan_create(arr, 1, None, res, None, ws, 0, 0, None, ctypes.byref(plan)) == _lib.LEXBFS_ENOWS
    assert not plan.value
    assert lib.lexbfs_batch_plan_launch(None, None) == _lib.LEXBFS_EINVAL
    lib.lexbfs_batch_plan_destroy(None)


def test_noalloc_argument_errors(lib):
    """The allocation-free entry point rejects bad arguments before any
    device work, and its fixed scratch covers the largest supported graph."""
    res = 0x20000
    assert lib.chordal_test_noalloc_max_bytes() >= lib.lexbfs_workspace_bytes(_lib.LEXBFS_MAX_N)
    assert lib.chordal_test_noalloc_max_bytes() < 8 << 20
    assert lib.chordal_test_noalloc(None, res, None, 0, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(_lib.LEXBFS_MAX_N + 1)
    assert lib.chordal_test_noalloc(ctypes.byref(g), res, None, 0, None) == _lib.LEXBFS_ETOOBIG
    g = fake_graph(100)
    assert lib.chordal_test_noalloc(ctypes.byref(g), None, None, 0, None) == _lib.LEXBFS_EINVAL
    assert lib.chordal_test_noalloc(ctypes.byref(g), res, None, _lib.LEXBFS_FLAG_VALIDATE, None) == _lib.LEXBFS_EINVAL
    g.reserved = 1
    assert lib.chordal_test_noalloc(ctypes.byref(g), res, None, 0, None) == _lib.LEXBFS_EINVAL


def test_workspace_sizes_grow(lib):
    sizes = [lib.lexbfs_workspace_bytes(n) for n in (0, 1, 64, 1000, 65536)]
    assert sizes == sorted(sizes) and sizes[0] > 0
    assert lib.lexbfs_workspace_bytes(65536) >= 10 * 4 * 65536


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert lib.lexbfs_strerror(code)
    assert lib.lexbfs_abi_version() >= 1


def test_python_constants_match_header():
    import re

    hdr = open(os.path.join(ROOT, "include", "lexbfs.h")).read()
    defs = {m.group(1): m.group(2) for m in re.finditer(r"#define\s+(LEXBFS_\w+)\s+\(?(-?(?:0x)?[0-9a-fA-F]+)u?\)?", hdr)}
    checked = 0
    for name, val in defs.items():
        if hasattr(_lib, name):
            assert getattr(_lib, name) == int(val, 0), name
            checked += 1
    assert checked >= 8 and "LEXBFS_FLAG_PER_STEP" in defs


def test_multi_sweep_argument_errors(lib):
    """LexBFS+ and the unit interval test reject bad arguments before any
    device work (the pointers below are never dereferenced)."""
    g = fake_graph(100)
    need = lib.lexbfs_plus_workspace_bytes(100, g.nnz)
    prev, order, ws, res = 0x40000, 0x50000, 0x60000, 0x70000
    assert need > lib.lexbfs_plus_workspace_bytes(50, g.nnz) > 0
    assert lib.lexbfs_plus_order(None, prev, order, None, None, ws, need, None) == _lib.LEXBFS_EINVAL
    assert lib.lexbfs_plus_order(ctypes.byref(g), None, order, None, None, ws, need, None) == _lib.LEXBFS_EINVAL
    assert lib.lexbfs_plus_order(ctypes.byref(g), prev, None, None, None, ws, need, None) == _lib.LEXBFS_EINVAL
    assert lib.lexbfs_plus_order(ctypes.byref(g), prev, order, None, None, ws, need - 1, None) == _lib.LEXBFS_ENOWS
    assert lib.lexbfs_plus_order(ctypes.byref(g), prev, order, None, None, None, need, None) == _lib.LEXBFS_ENOWS
    big = fake_graph(_lib.LEXBFS_MAX_N + 1)
    assert lib.lexbfs_plus_order(ctypes.byref(big), prev, order, None, None, ws, 1 << 40, None) == _lib.LEXBFS_ETOOBIG
    empty = fake_graph(0, nnz=0)
    assert lib.lexbfs_plus_order(ctypes.byref(empty), None, None, None, None, None, 0, None) == _lib.LEXBFS_OK
    # the bitset is not needed for a LexBFS+ sweep
    nobits = fake_graph(100)
    nobits.bits = None
    assert lib.lexbfs_plus_order(ctypes.byref(nobits), prev, order, None, None, ws, need - 1, None) == _lib.LEXBFS_ENOWS

    uneed = lib.unit_interval_workspace_bytes(100, g.nnz)
    assert uneed > need
    assert lib.unit_interval_test(ctypes.byref(g), None, None, ws, uneed, None) == _lib.LEXBFS_EINVAL
    assert lib.unit_interval_test(ctypes.byref(g), res, None, ws, uneed - 1, None) == _lib.LEXBFS_ENOWS
    assert lib.unit_interval_test(ctypes.byref(nobits), res, None, ws, uneed, None) == _lib.LEXBFS_EINVAL
    bad = fake_graph(100)
    bad.reserved = 3
    assert lib.unit_interval_test(ctypes.byref(bad), res, None, ws, uneed, None) == _lib.LEXBFS_EINVAL

    arr = (_lib.lexbfs_graph_t * 2)(fake_graph(10), fake_graph(20))
    bneed = lib.unit_interval_batch_workspace_bytes(arr, 2)
    assert bneed > 0 and lib.unit_interval_batch_workspace_bytes(None, 0) > 0
    assert lib.unit_interval_test_batch(arr, 2, None, None, ws, bneed, None) == _lib.LEXBFS_EINVAL
    assert lib.unit_interval_test_batch(arr, -1, res, None, ws, bneed, None) == _lib.LEXBFS_EINVAL
    assert lib.unit_interval_test_batch(arr, 0, None, None, None, 0, None) == _lib.LEXBFS_OK
    assert lib.unit_interval_test_batch(arr, 2, res, None, ws, bneed - 1, None) == _lib.LEXBFS_ENOWS
    arr = (_lib.lexbfs_graph_t * 2)(fake_graph(10), fake_graph(70000))
    assert lib.unit_interval_test_batch(arr, 2, res, None, ws, 1 << 40, None) == _lib.LEXBFS_ETOOBIG


def test_validate_argument_errors(lib):
    """lexbfs_validate rejects bad arguments before any device work; an
    empty graph needs no check (and no workspace)."""
    ws = 0x10000
    assert lib.lexbfs_validate(None, ws, 256, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(-1)
    assert lib.lexbfs_validate(ctypes.byref(g), ws, 256, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(_lib.LEXBFS_MAX_N + 1)
    assert lib.lexbfs_validate(ctypes.byref(g), ws, 256, None) == _lib.LEXBFS_ETOOBIG
    g = fake_graph(100, W=1)
    assert lib.lexbfs_validate(ctypes.byref(g), ws, 256, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(100)
    g.nnz = 1 << 31
    assert lib.lexbfs_validate(ctypes.byref(g), ws, 256, None) == _lib.LEXBFS_EINVAL
    g = fake_graph(100)
    assert lib.lexbfs_validate(ctypes.byref(g), None, 256, None) == _lib.LEXBFS_ENOWS
    assert lib.lexbfs_validate(ctypes.byref(g), ws, 255, None) == _lib.LEXBFS_ENOWS
    g = fake_graph(0, nnz=0)
    assert lib.lexbfs_validate(ctypes.byref(g), None, 0, None) == _lib.LEXBFS_OK
    assert lib.lexbfs_strerror(_lib.LEXBFS_EGRAPH) == b"graph violates the input contract"


def _device_code_object(tmp_path):
    """The gfx950 code object inside the built library (its offload bundle)."""
    llvm = "/opt/rocm/llvm/bin"
    bundler = os.path.join(llvm, "clang-offload-bundler")
    if not os.path.exists(bundler):
        pytest.skip("ROCm offload bundler not available")
    fatbin = tmp_path / "lib.hipfb"
    co = tmp_path / "lib.co"
    # Section contents into a file of their own: the library itself (loaded
    # in this process) is only read.
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", _lib.LIB_PATH, str(fatbin)], check=True)
    subprocess.run([bundler, "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fatbin}",
                    f"--output={co}", "--unbundle"], check=True)
    return llvm, co


def test_large_team_kernels_reserve_register_headroom(lib, tmp_path):
    """Kernels that run one 512- or 1,024-lane team per workgroup allocate at
    least 96 VGPRs (the v95 clobber at their entry): the 1,024-lane LexBFS
    kernel gave wrong orders when its allocation was exactly 88 registers with
    v84-v87 in use, and right ones with the same code at 96. The allocation
    is read from each kernel descriptor (COMPUTE_PGM_RSRC1, VGPR granules of 8)."""
    import struct

    llvm, co = _device_code_object(tmp_path)
    syms = subprocess.run([os.path.join(llvm, "llvm-readelf"), "-sW", str(co)], capture_output=True, text=True,
                          check=True).stdout
    secs = subprocess.run([os.path.join(llvm, "llvm-readelf"), "-SW", str(co)], capture_output=True, text=True,
                          check=True).stdout
    sections = []
    for line in secs.splitlines():
        m = re.match(r"\s*\[\s*\d+\]\s+(\S+)\s+\S+\s+([0-9a-f]+)\s+([0-9a-f]+)\s+([0-9a-f]+)", line)
        if m:
            sections.append((int(m.group(2), 16), int(m.group(3), 16), int(m.group(4), 16)))
    data = co.read_bytes()
    large = re.compile(r"(k_lexbfs_single|k_mcs_single|k_batch_large|k_finish_single)ILi(512|1024)E")
    checked = 0
    for line in syms.splitlines():
        f = line.split()
        if len(f) < 8 or not f[7].endswith(".kd") or not large.search(f[7]):
            continue
        addr = int(f[1], 16)
        sec = next(s for s in sections if s[0] <= addr < s[0] + s[2])
        kd = data[sec[1] + addr - sec[0]: sec[1] + addr - sec[0] + 64]
        rsrc1 = struct.unpack_from("<I", kd, 48)[0]
        vgprs = ((rsrc1 & 0x3F) + 1) * 8
        assert vgprs >= 96, (f[7], vgprs)
        checked += 1
    assert checked >= 15, checked  # every instantiation of these kernels at 512 and 1,024 lanes


def test_no_kernel_uses_the_top_of_an_88_register_allocation(lib, tmp_path):
    """No kernel of the library is built with 85-88 VGPRs (an allocation of
    88 with v84-v87 in use): the configuration that gave wrong LexBFS orders
    with otherwise correct machine code. Counts from the code object's
    kernel metadata."""
    llvm, co = _device_code_object(tmp_path)
    notes = subprocess.run([os.path.join(llvm, "llvm-readelf"), "--notes", str(co)], capture_output=True, text=True,
                           check=True).stdout
    counts = {}
    for block in re.split(r"\n\s+- \.", notes):
        name = re.search(r"\.name:\s+(\S+)", block)
        vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
        if name and vgpr:
            counts[name.group(1)] = int(vgpr.group(1))
    assert len(counts) >= 40, len(counts)
    bad = {k: v for k, v in counts.items() if 85 <= v <= 88}
    assert not bad, bad

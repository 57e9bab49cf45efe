"""The C ABI of librsaw (include/rsaw.h) on the CPU: the built library loads,
exports every declared symbol, and rejects invalid configurations with the
documented status before touching a device.  Also checks that the product
package has no path into the oracle and no CPU fallback."""
import ctypes as C
import os
import re

import pytest

import paper_1704_04381_amd as rs

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(rs.LIB_PATH):
        pytest.skip("librsaw.so not built (run __graft_entry__.build())")
    return rs.load()


def test_header_declarations_match_exports():
    hdr = open(os.path.join(REPO, "include", "rsaw.h")).read()
    declared = set(re.findall(r"^[A-Za-z_][\w \*]*?\b(rsaw_\w+)\s*\(", hdr, re.M))
    assert declared == set(rs.EXPORTS), declared
    lib = _lib()
    for name in declared:
        assert hasattr(lib, name), name


def test_summary_struct_layout():
    # the ctypes mirror must match the C struct size: 19 eight-byte fields,
    # three 16-byte exact sums, two int32
    assert rs.SUMMARY_BYTES == 19 * 8 + 3 * 16 + 8


BAD = [
    (dict(geometry="lattice", N=0, k=6), 1),
    (dict(geometry="lattice", N=70000, k=6), 1),
    (dict(geometry="lattice", N=16, k=5), 1),
    (dict(geometry="lattice", N=16, k=6, coord="f64"), 1),
    (dict(geometry="lattice", N=29, k=6, exact_w=True), 3),
    (dict(geometry="lattice", N=16385, k=6), 2),
    (dict(geometry="real", N=16, k=0), 1),
    (dict(geometry="real", N=16, k=65), 1),
    (dict(geometry="real", N=16, k=8, coord="i32"), 1),
    (dict(geometry="real", N=16, k=8, bond_length=0.0), 1),
    (dict(geometry="real", N=16, k=8, bead_diameter=-1.0), 1),
    (dict(geometry="real", N=16, k=8, bond_length=float("nan")), 1),
    (dict(geometry="real", N=16, k=8, exact_w=True), 1),
    (dict(geometry="real", N=16385, k=8), 2),
    (dict(geometry="lattice26", N=16, k=6), 1),
    (dict(geometry="lattice26", N=16, k=26, coord="f64"), 1),
    (dict(geometry="lattice26", N=15, k=26, exact_w=True), 3),
    (dict(geometry="lattice26", N=16385, k=26), 2),
    (dict(geometry="lattice", N=16, k=26), 1),
    (dict(geometry=7, N=16, k=6), 1),
    (dict(geometry="lattice", N=16, k=6, hist_bins=-1), 1),
    (dict(geometry="lattice", N=16, k=6, hist_bins=300), 2),
    (dict(geometry="lattice", N=16, k=6, n_chains=1 << 32), 1),
]


@pytest.mark.parametrize("kw,status", BAD)
def test_invalid_configs_rejected(kw, status):
    lib = _lib()
    kw = dict(kw)
    n = kw.pop("n_chains", 10)
    cfg = rs.make_config(kw.pop("geometry"), kw.pop("N"), kw.pop("k"), n, 1, **kw)
    got = lib.rsaw_gen_chains(C.byref(cfg), None, None, None, None, None)
    assert got == status, (got, lib.rsaw_last_error())
    assert lib.rsaw_last_error().decode() != ""
    assert lib.rsaw_status_string(got).decode() not in ("", "unknown status")


def test_null_arguments():
    lib = _lib()
    assert lib.rsaw_gen_chains(None, None, None, None, None, None) == 1
    cfg = rs.make_config("lattice", 16, 6, 10, 1)
    assert lib.rsaw_gen_chains_sync(C.byref(cfg), None, None, None, None, None) == 1
    cfg.flags = 0x80
    assert lib.rsaw_gen_chains(C.byref(cfg), None, None, None, None, None) == 1
    assert lib.rsaw_version() >= 100
    assert lib.rsaw_status_string(99).decode() == "unknown status"


def test_batch_argument_errors():
    lib = _lib()
    assert lib.rsaw_gen_batch(None, None, 0, None, None, None, None) == 0
    assert lib.rsaw_gen_batch(None, None, -1, None, None, None, None) == 1
    assert lib.rsaw_gen_batch(None, None, 3, None, None, None, None) == 1
    good = rs.make_config("lattice", 16, 6, 10, 1)
    bad = rs.make_config("real", 16, 65, 10, 1)
    arr = (rs.rsaw_config * 3)(good, bad, good)
    assert lib.rsaw_gen_batch(arr, None, 3, None, None, None, None) == 1
    assert "ensemble 1" in lib.rsaw_last_error().decode()


def test_server_argument_errors():
    lib = _lib()
    h = C.c_void_p()
    bad = rs.rsaw_server_params(1 << 20, 0, 1)
    assert lib.rsaw_server_create(C.byref(bad), 0, C.byref(h)) == 1
    bad = rs.rsaw_server_params(1 << 20, 8, 17)
    assert lib.rsaw_server_create(C.byref(bad), 0, C.byref(h)) == 1
    assert lib.rsaw_server_create(None, 0, None) == 1
    assert lib.rsaw_server_submit(None, None, None) == 1
    assert lib.rsaw_server_wait(None, 1, None, None) == 1
    lib.rsaw_server_destroy(None)


def test_kernel_timing_switch_without_launches():
    lib = _lib()
    assert lib.rsaw_kernel_timing(1) == 0
    assert rs.kernel_time() == (0.0, 0)
    assert lib.rsaw_kernel_timing(0) == 0
    assert lib.rsaw_kernel_time(None, None) == 0


def test_no_cpu_fallback_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    _lib()
    with pytest.raises(rs.RsawError):
        rs.gen_chains("lattice", 16, 6, 10, 1)


def test_product_package_never_touches_the_oracle():
    pkg = os.path.join(REPO, "paper_1704_04381_amd")
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(root, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b|rsaw_oracle|\boro_|"
                                     r"import_module\(.oracle", txt, re.M), f


def test_workspace_size_query_on_host():
    """rsaw_workspace_size is host-only: it needs no GPU and reports the
    per-chain reduction arrays (26 B per chain) unless the caller supplies
    them, the small fixed cells, and the HBM bead planes of long hard-sphere
    chains (3 N doubles per resident block, at most 2048 blocks)."""
    import ctypes as C

    M = 10**7
    cfg = rs.make_config("lattice", 64, 6, M, 1, coord="i16", hist_bins=256)
    full = rs.workspace_size(cfg)
    assert 26 * M <= full <= 26 * M + (1 << 20)
    o = rs.rsaw_chain_out()
    o.log_w = o.r2 = o.rg2 = o.n_grown = 1  # any non-NULL address: not dereferenced
    supplied = rs.workspace_size(cfg, o)
    assert supplied < (1 << 20) and full - supplied >= 26 * M
    assert rs.workspace_size(cfg, None, reduce=False) < (1 << 18)  # fixed cells and block partials
    real = rs.workspace_size(rs.make_config("real", 2000, 8, 5000, 1), None, reduce=False)
    assert 2048 * 3 * 2000 * 8 <= real <= 2048 * 3 * 2000 * 8 + (1 << 18)
    small = rs.workspace_size(rs.make_config("real", 1536, 8, 5000, 1), None, reduce=False)
    assert small < (1 << 18)  # LDS planes up to N = 1536
    with pytest.raises(rs.RsawError) as e:
        rs.workspace_size(rs.make_config("lattice26", 16, 6, 10, 1))
    assert e.value.status == 1
    lib = rs.load()
    assert lib.rsaw_workspace_size(C.byref(cfg), None, 1, None) == 1


def test_header_is_plain_c99(tmp_path):
    """include/rsaw.h compiles as strict C99 (no C++ or torch types leak into
    the boundary)."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "use_header.c"
    src.write_text('#include "rsaw.h"\nint main(void) { rsaw_config c; rsaw_mapping m; (void)c; (void)m; return 0; }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-I", inc,
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_set_workspace_argument_errors():
    """rsaw_set_workspace checks alignment and the minimum size on the host
    before any device call; NULL unbinds."""
    lib = _lib()
    assert lib.rsaw_set_workspace(C.c_void_p(0x1001), 1 << 20, None) == 1
    assert "aligned" in lib.rsaw_last_error().decode()
    assert lib.rsaw_set_workspace(C.c_void_p(0x100000), 64, None) == 1
    assert "at least" in lib.rsaw_last_error().decode()
    # the smallest workspace is that of an empty reducing call
    least = rs.workspace_size(rs.make_config("lattice", 1, 6, 0, 1))
    assert 0 < least <= 4096


def test_fp64_check_argument_errors():
    lib = _lib()
    assert lib.rsaw_fp64_check(None, None, None, None, 0, None) == 0
    assert lib.rsaw_fp64_check(None, None, None, None, 5, None) == 1

"""The C-ABI library builds, loads and exports every declared symbol; the
host-only entry points and the argument checks work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2511_09546_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)
    keep = []
    for nm in names:
        if nm in ("sizeof", "defined") or nm in keep:
            continue
        keep.append(nm)
    return keep


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2511_09546_amd import build
        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared("ipeps.h") + _declared("ipeps_debug.h")
    assert set(binding.API_FUNCTIONS) <= set(declared)
    for name in declared:
        assert hasattr(lib, name), name
    for name in binding.API_FUNCTIONS + binding.DEBUG_FUNCTIONS:
        assert name in declared


def test_host_only_entry_points(lib):
    assert binding.strerror(binding.EINVAL) == "invalid argument"
    assert lib.ipeps_version().decode().startswith("ipeps")
    o = binding.default_opts()
    assert o.prec == binding.FP64 and o.grad_K == 20
    assert o.svd_cutoff == 1e-12 and o.svd_tol == 1e-13
    assert lib.ipeps_env_size(2, 2, 3, 10) == 4 * 4 * 100 + 4 * 4 * 10 * 9 * 10


def test_argument_checks_before_any_device_call(lib):
    A = np.zeros((1, 1, 2, 3, 3, 3, 3))
    h = ctypes.c_void_p()
    dp = A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # chi < D^2, bad sizes, null pointers: rejected on the host
    assert lib.ctm_init(ctypes.byref(h), 1, 1, 2, 3, 8, dp, None, None) == -1
    assert lib.ctm_init(ctypes.byref(h), 0, 1, 2, 3, 9, dp, None, None) == -1
    assert lib.ctm_init(None, 1, 1, 2, 3, 9, dp, None, None) == -1
    A[0, 0, 0, 0, 0, 0, 0] = np.nan
    assert lib.ctm_init(ctypes.byref(h), 1, 1, 2, 3, 9, dp, None, None) == -1
    # an option outside its range (grad_checkpoint is 0 or 1)
    A[0, 0, 0, 0, 0, 0, 0] = 0.0
    o = binding.default_opts()
    o.grad_checkpoint = 2
    assert lib.ctm_init(ctypes.byref(h), 1, 1, 2, 3, 9, dp, ctypes.byref(o),
                        None) == -1
    assert lib.ctm_converge(None, 1e-10, 10, None, None) == -1
    assert lib.precond_apply(None, None, 1.0, 0.0, 1, None, None, None) == -1
    lib.ctm_free(None)


def test_noalloc_scratch_size_and_estimate(lib):
    """The scratch size the binding states is the header's, and the host-only
    working-set estimate admits the D=6, chi=72 state and refuses chi=100."""
    import re
    hdr = open(os.path.join(ROOT, "include", "ipeps.h")).read()
    m = re.search(r"#define IPEPS_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)",
                  hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == \
        binding.NOALLOC_SCRATCH_BYTES
    cap = binding.NOALLOC_SCRATCH_BYTES
    need = binding.noalloc_bytes(1, 1, 2, 6, 72)
    # three chi^2 D^4 half-ring blocks dominate
    assert 3 * 8 * 72 ** 2 * 6 ** 4 < need <= cap
    assert binding.noalloc_bytes(1, 1, 2, 6, 100) > cap
    assert binding.noalloc_bytes(0, 1, 2, 6, 72) == 0
    assert lib.precond_apply_dev_noalloc(None, None, 1e-4, 0.0, 1, None,
                                         None, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the C structs have the header's size and field
    offsets (compiled with the host C compiler)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_2511_09546_amd import binding
    structs = {"ipeps_opts": binding.Opts, "ipeps_term": binding.Term,
               "ipeps_lbfgs_params": binding.LbfgsParams,
               "ipeps_lbfgs_info": binding.LbfgsInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>',
             '#include "ipeps.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", '
                         f'offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)

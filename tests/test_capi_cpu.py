"""CPU checks of the C ABI: the built library loads and exports every function
include/resalloc.h declares; calls that need no device behave as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "resalloc.h")
LIB = os.path.join(ROOT, "paper_2104_00282_amd", "libresalloc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ra_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libresalloc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    for fn in ("ra_create", "ra_destroy", "ra_problem_create", "ra_dual_eval", "ra_solve",
               "ra_get_allocation", "ra_status_string", "ra_last_error"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        getattr(lib, f)


def test_binding_names_match_header():
    from paper_2104_00282_amd import _capi
    assert set(_capi.PROTOTYPES) == set(declared_functions())


def test_binding_structs_match_header_layout(tmp_path):
    """The ctypes mirrors of ra_solve_opts and ra_solve_info have the C
    compiler's size and field offsets (a field added to one side only would
    shift every later field)."""
    from paper_2104_00282_amd import _capi
    structs = (_capi.ra_solve_opts, _capi.ra_solve_info)
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "resalloc.h"',
             "int main(void) {"]
    for st in structs:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (st.__name__, st.__name__))
        for f, _ in st._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));'
                         % (st.__name__, f, st.__name__, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", exe])
    got = dict(l.split() for l in subprocess.check_output([exe], text=True).splitlines())
    for st in structs:
        assert int(got[st.__name__]) == ctypes.sizeof(st), st.__name__
        for f, _ in st._fields_:
            assert int(got["%s.%s" % (st.__name__, f)]) == getattr(st, f).offset, (st, f)
    # and every field the header declares is mirrored, in order
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for st in structs:
        body = re.search(r"typedef struct \{([^}]*)\}\s*%s;" % st.__name__, text).group(1)
        names = re.findall(r"\b(\w+)\s*;", body)
        assert names == [f for f, _ in st._fields_], st.__name__


def test_status_strings_and_defaults(lib):
    import paper_2104_00282_amd as ra
    assert ra.ra_status_string(ra.RA_OK) == "ok"
    assert ra.ra_status_string(ra.RA_ENOTCONV) == "not converged"
    assert ra.ra_status_string(99) == "unknown status"
    o = ra.ra_solve_opts_default()
    assert (o.tol_rel, o.max_iter, o.lbfgs_mem, o.method, o.init, o.use_graph, o.max_evals,
            o.stall_evals, o.init_step, o.tol_abs, o.device_loop, o.stall_restarts,
            o.warm_stall_restarts, o.warm_stall_evals) == \
        (1e-6, 500, 10, 0, 0, 1, 0, 0, 0.0, 0.0, 0, 0, -1, 0)


def test_null_arguments_rejected_without_device(lib):
    import paper_2104_00282_amd as ra
    L = ra._capi.lib()
    assert L.ra_create(None, 0, None) == ra.RA_EINVAL
    assert L.ra_destroy(None) == ra.RA_OK
    assert L.ra_problem_destroy(None) == ra.RA_OK
    assert L.ra_dual_eval(None, None, None, None, None, None, None, None, None) == ra.RA_EINVAL
    assert L.ra_solve(None, None, None, None, None) == ra.RA_EINVAL
    assert L.ra_get_allocation(None, None, None, None) == ra.RA_EINVAL
    assert L.ra_set_kernel_timing(None, 1) == ra.RA_EINVAL
    assert L.ra_last_error(None) == b""
    assert L.ra_batch_set_shape(None, 2048, None, 0) == ra.RA_EINVAL
    assert L.ra_batch_tuning(None, None, 0, None) == ra.RA_EINVAL


def test_create_without_gpu_reports_device_error():
    """In a container without a GPU, ra_create fails cleanly (no crash)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_2104_00282_amd as ra
    with pytest.raises(ra.RAError) as e:
        ra.ra_create(0)
    assert e.value.status == ra.RA_EDEVICE

"""The C-ABI library loads and exports every symbol its header declares; host
logic that needs no GPU. No compute calls are made here."""

import ctypes as ct
import os
import re
import subprocess

import pytest

from paper_1805_01559_amd import ot_assoc as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ot_assoc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libot_assoc.so not built")
    return A.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert names, "no declarations parsed"
    assert set(names) == set(A.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ot_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    fields = ["sizeof(ot_cost_desc)", "sizeof(ot_assoc_options)", "sizeof(ot_assoc_result)",
              "offsetof(ot_cost_desc, geom)", "offsetof(ot_assoc_result, seconds)",
              "offsetof(ot_assoc_options, batch_tune)", "sizeof(ot_serve_options)",
              "offsetof(ot_serve_options, keep_layouts)", "sizeof(ot_request)", "offsetof(ot_request, layout_key)",
              "offsetof(ot_request, user_tag)", "sizeof(ot_completion)", "offsetof(ot_completion, result)",
              "offsetof(ot_completion, t_done)", "offsetof(ot_assoc_options, persistent)",
              "sizeof(ot_eval_result)", "offsetof(ot_eval_result, devices_overloaded)",
              "sizeof(ot_adaptive_result)", "offsetof(ot_adaptive_result, delta)",
              "offsetof(ot_assoc_options, check_every)", "offsetof(ot_assoc_options, workspace)",
              "offsetof(ot_assoc_options, workspace_bytes)", "offsetof(ot_assoc_options, snapshot_k_split)"]
    fmt = " ".join(["%zu"] * len(fields))
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ot_assoc.h"\n'
                   'int main(void){printf("' + fmt + '\\n", ' + ", ".join(fields) + ');return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    want = [ct.sizeof(A.ot_cost_desc), ct.sizeof(A.ot_assoc_options), ct.sizeof(A.ot_assoc_result),
            A.ot_cost_desc.geom.offset, A.ot_assoc_result.seconds.offset, A.ot_assoc_options.batch_tune.offset,
            ct.sizeof(A.ot_serve_options), A.ot_serve_options.keep_layouts.offset, ct.sizeof(A.ot_request),
            A.ot_request.layout_key.offset, A.ot_request.user_tag.offset, ct.sizeof(A.ot_completion),
            A.ot_completion.result.offset, A.ot_completion.t_done.offset, A.ot_assoc_options.persistent.offset,
            ct.sizeof(A.ot_eval_result), A.ot_eval_result.devices_overloaded.offset,
            ct.sizeof(A.ot_adaptive_result), A.ot_adaptive_result.delta.offset,
            A.ot_assoc_options.check_every.offset, A.ot_assoc_options.workspace.offset,
            A.ot_assoc_options.workspace_bytes.offset, A.ot_assoc_options.snapshot_k_split.offset]
    assert got == want


def test_default_options(lib):
    o = A.ot_assoc_default_options()
    assert (o.device, o.precision, o.polish_iters, o.chunk, o.use_graphs, o.batch_tune, o.persistent,
            o.check_every, o.workspace, o.workspace_bytes, o.snapshot_k_split) == (0, A.OT_PREC_FP32, 1, 8, 1, 1, 1,
                                                                                    1, None, 0, 1)
    s = A.ot_serve_default_options()
    assert (s.polish_iters, s.sweep_waves, s.rows_per_part, s.max_slots, s.budget_bytes) == (1, 8, 128, 0, 0.0)


def test_batch_and_serve_argument_errors_without_a_device(lib):
    assert lib.ot_assoc_solve_batch(None, 1, None, None, None, None, 1e-6, 10, None) == A.OT_EINVAL
    assert lib.ot_assoc_batch_potentials(None, 0, None, None, 0) == A.OT_EINVAL
    assert lib.ot_assoc_batch_plan(None, 0, None, 0, 0) == A.OT_EINVAL
    assert lib.ot_serve_submit(None, None, None) == A.OT_EINVAL
    assert lib.ot_serve_progress(None, None, 0, None) == A.OT_EINVAL
    assert lib.ot_serve_counts(None, None, None, None, None) == A.OT_EINVAL
    # bad options are rejected before any device is touched
    o = A.ot_serve_default_options()
    o.rows_per_part = 100
    with pytest.raises(A.OTError):
        A.ot_serve_create(o)
    o = A.ot_serve_default_options()
    o.sweep_waves = 6
    with pytest.raises(A.OTError):
        A.ot_serve_create(o)
    lib.ot_serve_destroy(None)
    assert lib.ot_serve_now() > 0.0


def test_workspace_size_without_a_device(lib):
    # pure host arithmetic: grows with the instance, 256-byte granular, rejects bad sizes
    small = A.ot_assoc_workspace_size(1000, 50)
    big = A.ot_assoc_workspace_size(20000, 400)
    assert 0 < small < big and small % 256 == 0 and big % 256 == 0
    # at least the potentials (two parities), marginals and the scratch region
    assert big >= 8 * (2 * 20000 + 2 * 400 + 20000 + 400 + 2 * (20000 + 400))
    for I, J in [(0, 10), (10, 0), (10, 5000)]:
        with pytest.raises(A.OTError):
            A.ot_assoc_workspace_size(I, J)
    assert A.ot_assoc_device_allocations() >= 0
    # the no-allocation solve keeps a handle's buffers for 32768 x 512 in its fixed 9 MiB array
    assert A.ot_assoc_workspace_size(32768, 512) <= 9 << 20
    # a workspace size without a workspace is rejected before any device is touched
    o = A.ot_assoc_default_options()
    o.workspace_bytes = 4096
    with pytest.raises(A.OTError) as e:
        A.ot_assoc_create(10, 10, o)
    assert e.value.status == A.OT_EINVAL
    o = A.ot_assoc_default_options()
    o.check_every = -1
    with pytest.raises(A.OTError):
        A.ot_assoc_create(10, 10, o)


def test_argument_errors_without_a_device(lib):
    # invalid sizes are rejected before any device is touched
    with pytest.raises(A.OTError) as e:
        A.ot_assoc_create(0, 10)
    assert e.value.status == A.OT_EINVAL
    with pytest.raises(A.OTError) as e:
        A.ot_assoc_create(10, 5000)
    assert e.value.status == A.OT_EINVAL
    # NULL handles are rejected, destroy is NULL-safe
    assert lib.ot_assoc_solve(None, None, None, None, 0.1, 1e-6, 10, 0, None) == A.OT_EINVAL
    assert lib.ot_assoc_plan(None, None, 0, 0) == A.OT_EINVAL
    lib.ot_assoc_destroy(None)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1805_01559_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in text.lower().replace("# the oracle", ""), fn

"""The C-ABI library: it loads, exports every entry point include/orrb.h declares, and
the binding's struct layouts match the header (CPU only: no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "orrb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(orrb_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1906_11633_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liborrb.so not built")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1906_11633_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_struct_sizes_match_header():
    """Compile a tiny C program against the header and compare struct sizes/offsets
    with the ctypes declarations."""
    import subprocess
    import tempfile
    from paper_1906_11633_amd import _lib as L
    structs = {"orrb_layout_desc": L.LayoutDesc, "orrb_tuning": L.Tuning, "orrb_layout_info": L.LayoutInfo,
               "orrb_scenes": L.Scenes, "orrb_cameras": L.Cameras, "orrb_params": L.Params, "orrb_outputs": L.Outputs,
               "orrb_track": L.Track, "orrb_kernel_times": L.KernelTimes}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "s.c"), os.path.join(d, "s")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_create_without_gpu_reports_error(lib):
    """With no GPU visible, orrb_create fails with a status and a message instead of
    aborting."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = lib.orrb_create(0, C.byref(h))
    assert st != 0
    assert lib.orrb_last_error()
    assert not h.value


def test_null_arguments_rejected(lib):
    """Host validation returns ORRB_ERR_INVALID_ARGUMENT for NULL handles before any
    device work."""
    assert lib.orrb_create(0, None) == 1
    mid = C.c_int32()
    assert lib.orrb_add_mesh(None, None, None, 3, None, 1, C.byref(mid)) == 1
    assert lib.orrb_render_batch(None, None, None, None, None, None, None, 0, None) == 1
    assert lib.orrb_layout_info_get(None, None) == 1
    assert lib.orrb_wait_timeouts(None, None) == 1
    assert lib.orrb_validate_batch(None, None, None, None, None, None, None) == 1
    lib.orrb_destroy(None)
    lib.orrb_layout_destroy(None)


def test_paper_context_fixture():
    """The paper's printed throughput (Sec. 5, Tables 2-3) used as bench context."""
    import json
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_throughput.json")))
    assert d["table2_gpu_scaling"] == {"1": 1342, "2": 2870, "3": 3395, "4": 3514}
    t3 = [d["table3_render_servers_on_8_gpus"][k] for k in sorted(d["table3_render_servers_on_8_gpus"], key=int)]
    assert t3 == sorted(t3) and t3[0] == 736 and t3[-1] == 3438


def test_stat_words_match_header():
    """The binding's names of the per-call counters follow the header's word indices."""
    from paper_1906_11633_amd import _lib as L
    text = open(HEADER).read()
    words = {m.group(1).lower(): int(m.group(2)) for m in re.finditer(r"#define ORRB_STAT_([A-Z_]+)\s+(\d+)", text)}
    assert int(re.search(r"#define ORRB_STATS_WORDS\s+(\d+)", text).group(1)) == L.STATS_WORDS
    assert int(re.search(r"#define ORRB_POST_WORDS\s+(\d+)", text).group(1)) == L.POST_WORDS
    assert C.sizeof(L.Track) == L.TRACK_BYTES
    header_order = [k for k, _ in sorted(words.items(), key=lambda kv: kv[1])]
    assert [v for _, v in sorted(words.items(), key=lambda kv: kv[1])] == list(range(len(words)))
    expect = {"wait_timeouts": "wait_timeouts", "bin_overflow_frames": "bin_overflow",
              "survivor_resetup_frames": "survivor_resetup", "near_vertices": "near_vertices",
              "guard_vertices": "guard_vertices", "tiled_extra_flushes": "tiled_extra_flush",
              "invalid_state": "invalid_state"}
    assert [expect[n] for n in L.STAT_NAMES] == header_order

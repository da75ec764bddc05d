"""CPU checks of the library boundary: libtrk.so loads, exports every entry
point declared in include/trk.h, its structs match the binding's, and host-side
validation rejects bad configurations before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from gen import TINY, MU200, make_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trk.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|int64_t|void|const char\*)\s+(trk_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2501_05520_amd import trk
    lib = trk.lib()
    declared = _declared()
    assert set(declared) == set(trk.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", trk.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (trk_\w+)$", out, re.M))
    assert set(declared) <= exported
    for name in declared:
        assert hasattr(lib, name)


def test_struct_layouts_match_header(tmp_path):
    from paper_2501_05520_amd import trk
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "trk.h"\n'
                   'int main(){printf("%zu %zu %zu %zu\\n", sizeof(trk_config), sizeof(trk_event_info),'
                   ' offsetof(trk_config, max_hits), offsetof(trk_config, max_events));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(trk.trk_config), ctypes.sizeof(trk.trk_event_info),
            trk.trk_config.max_hits.offset, trk.trk_config.max_events.offset]
    assert list(map(int, got)) == want


def test_strerror():
    from paper_2501_05520_amd import trk
    assert trk.trk_strerror(0) == "ok"
    assert "capacity" in trk.trk_strerror(-3)
    assert "deadline" in trk.trk_strerror(-7)
    assert "shutting down" in trk.trk_strerror(-8)
    assert trk.trk_strerror(-99) == "unknown status"


@pytest.mark.parametrize("field,value", [("abi_version", 99), ("emb_hidden", 100), ("emb_dim", 17),
                                         ("filt_hidden", 48), ("gnn_hidden", 64), ("k_max", 0),
                                         ("radius", -1.0), ("precision", 7), ("precision", -1), ("max_hits", 0),
                                         ("precision", 2), ("precision", 3), ("precision", 9)])
def test_create_rejects_bad_config(field, value):
    # (the FP8 precisions are rejected for the tiny widths, 64 not being a multiple of 128)
    from paper_2501_05520_amd import trk
    cfg = trk.make_config(TINY, "fp32", max_hits=1000)
    setattr(cfg, field, value)
    blob = trk.pack_weights(TINY, make_weights(TINY, 0))
    h = ctypes.c_void_p()
    rc = trk.lib().trk_create(ctypes.byref(cfg), blob, len(blob), 0, ctypes.byref(h))
    assert rc == -1 and not h.value


def test_entry_points_reject_null_context():
    from paper_2501_05520_amd import trk
    L = trk.lib()
    n = ctypes.c_int64()
    assert L.trk_embed(None, None, 0, None, None) == -1
    assert L.trk_event(None, None, 0, None, None, None) == -1
    assert L.trk_build_graph(None, None, 0, None, None, 0, ctypes.byref(n), None, None) == -1
    L.trk_destroy(None)


@pytest.mark.parametrize("cfg", [TINY, MU200], ids=["tiny", "mu200"])
def test_weight_blob_size(cfg):
    from paper_2501_05520_amd import trk
    nets = make_weights(cfg, 0)
    blob = trk.pack_weights(cfg, nets)
    n_float = sum(w.size + b.size for layers in nets.values() for w, b in layers)
    assert len(blob) == 64 + 4 * n_float
    hdr = np.frombuffer(blob[:64], np.uint32)
    assert hdr[0] == trk.TRK_WEIGHTS_MAGIC and hdr[2] == cfg.emb_hidden and hdr[8] == cfg.gnn_iters

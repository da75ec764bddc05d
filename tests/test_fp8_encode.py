"""The host E4M3 encoder used for FP8 weights (csrc/host_quant.h), built with g++,
against torch's float8_e4m3fn conversion (round to nearest even) on values
clamped to +-448 (the encoder saturates), and its power-of-two tensor scale
against its definition."""
import math
import os
import subprocess

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))


def test_e4m3_encoder(tmp_path):
    exe = tmp_path / "fp8_encode"
    subprocess.run(["g++", "-std=c++17", "-O1", os.path.join(HERE, "native", "fp8_encode_test.cpp"), "-o", str(exe)],
                   check=True)
    rng = np.random.default_rng(0)
    # every code point, the midpoints between neighbours (ties), random values over
    # the whole range and beyond, subnormals, zeros and saturation
    codes = torch.arange(0, 256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    finite = np.sort(codes[np.isfinite(codes) & (codes >= 0)])
    mids = (finite[1:] + finite[:-1]) / 2
    vals = np.concatenate([finite, -finite, mids, -mids, rng.normal(0, 1, 4000) * 10.0 ** rng.uniform(-4, 3, 4000),
                           [0.0, -0.0, 447.9, 448.0, 460.0, 464.0, 1e4, -1e4, 2.0 ** -10, 3 * 2.0 ** -11]])
    vals = vals.astype(np.float32)
    inp = "\n".join(f"{x:08x}" for x in vals.view(np.uint32)) + "\n"
    r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    lines = r.stdout.split("\n")
    got = np.array([int(t) for t in lines[:vals.size]], dtype=np.uint8)
    want = torch.from_numpy(np.clip(vals, -448, 448)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # negative zero encodes as 0x80 in both
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, [(float(vals[i]), int(got[i]), int(want[i])) for i in bad[:10]]
    scale = float(lines[vals.size].split()[1])
    amax = float(np.abs(vals).max())
    assert scale == 2.0 ** math.floor(math.log2(448.0 / amax))
    assert amax * scale <= 448.0 < 2 * amax * scale

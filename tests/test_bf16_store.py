"""FP32 -> BF16 rounding of the stored operators (host build of the device helper).

Round to nearest even on finite values; NaN stays NaN (no wrap to zero or to
infinity), infinities stay infinities, values beyond the largest bfloat16 round
to infinity.  Finite cases are compared with the oracle's rounding.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.learned import bf16_round

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("bf16") / "bf16_store_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", os.path.join(HERE, "bf16_store_check.cpp"),
                    "-o", out], check=True, capture_output=True)
    return out


def run(checker, bits):
    txt = "\n".join(f"{int(b):08x}" for b in bits) + "\n"
    r = subprocess.run([checker], input=txt, capture_output=True, text=True, check=True)
    return np.array([int(x, 16) for x in r.stdout.split()], dtype=np.uint32)


def test_nan_inf_and_overflow(checker):
    bits = [0x7FC00000, 0x7FFF8000, 0x7FFFFFFF, 0xFFFF8000, 0xFFFFFFFF, 0x7F800001, 0xFF800001,
            0x7F800000, 0xFF800000, 0x7F7FFFFF, 0xFF7FFFFF]
    out = run(checker, bits)
    for b, h in zip(bits[:7], out[:7]):
        assert (h & 0x7F80) == 0x7F80 and (h & 0x007F) != 0, (hex(b), hex(h))  # NaN
        assert (h >> 15) == (b >> 31)  # sign kept
    assert list(out[7:9]) == [0x7F80, 0xFF80]  # infinities
    assert list(out[9:11]) == [0x7F80, 0xFF80]  # max float rounds to infinity


def test_finite_values_round_to_nearest_even(checker):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-30, 30, 2000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 2 ** -130]]).astype(np.float32)
    bits = x.view(np.uint32)
    out = run(checker, bits)
    ref = bf16_round(x.astype(np.float64)).to("cpu").numpy().astype(np.float32).view(np.uint32) >> 16
    assert np.array_equal(out, ref.astype(np.uint32))

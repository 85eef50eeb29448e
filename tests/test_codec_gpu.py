"""The gfx950 hardware conversions used by the kernels against the oracle's
codecs: every e4m3 code decoded, and FP32 -> e4m3 / BF16 rounding bit-exact on
edge cases and random FP32 bit patterns (both sides decide from the same exact
FP32 value).  NaN inputs are out of scope (the FP8 encoder saturates them)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C

pytestmark = pytest.mark.gpu


def _edge_values():
    v = [0.0, -0.0, 2.0 ** -10, 1.5 * 2.0 ** -10, 2.0 ** -9, 2.0 ** -7, 2.0 ** -6, 1.0, 1.0625, 1.1875,
         447.0, 448.0, 455.0, 456.0, 460.0, 463.99, 464.0, 480.0, 1e6, 3.0e38, 1e-30]
    return np.array(v + [-x for x in v], dtype=np.float32)


def _random_fp32(n, seed, lo_exp=-40, hi_exp=40):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    e = np.floor(np.log2(np.maximum(np.abs(x.astype(np.float64)), 1e-300)))
    return x[(e >= lo_exp) & (e <= hi_exp)]


def test_fp8_decode_all_codes(gpu_handle):
    codes = np.arange(256, dtype=np.uint8)
    finite = codes[(codes & 0x7F) != 0x7F]
    t = torch.from_numpy(finite.reshape(1, -1)).cuda()
    got = C.decode(t, torch.ones(1, device="cuda"), h=gpu_handle).double().cpu().numpy()[0]
    assert np.array_equal(got, oracle.decode_e4m3(finite))


def test_fp8_encode_matches_oracle(gpu_handle):
    x = np.concatenate([_edge_values(), _random_fp32(1 << 21, 1, -12, 9),
                        np.random.default_rng(2).uniform(-470, 470, 1 << 18).astype(np.float32)])
    t = torch.from_numpy(x.reshape(1, -1)).cuda()
    got = C.encode(t, C.FP8, h=gpu_handle).cpu().numpy()[0]
    ref = oracle.encode_e4m3(x.astype(np.float64))
    bad = np.nonzero(oracle.decode_e4m3(got) != oracle.decode_e4m3(ref))[0]
    assert bad.size == 0, [(float(x[i]), int(got[i]), int(ref[i])) for i in bad[:8]]


def test_bf16_encode_matches_oracle(gpu_handle):
    x = np.concatenate([_edge_values(), _random_fp32(1 << 21, 3, -126, 127)])
    t = torch.from_numpy(x.reshape(1, -1)).cuda()
    got = C.encode(t, C.BF16, h=gpu_handle).view(torch.int16).cpu().numpy()[0].view(np.uint16)
    ref = oracle.encode_bf16(x.astype(np.float64))
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(float(x[i]), hex(got[i]), hex(ref[i])) for i in bad[:8]]


def test_fp8_encode_with_row_scale(gpu_handle):
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((5, 333)) * 20).astype(np.float32)
    s = (np.abs(x).max(1) / 448.0).astype(np.float32)
    got = C.encode(torch.from_numpy(x).cuda(), C.FP8, torch.from_numpy(s).cuda(), h=gpu_handle).cpu().numpy()
    # the kernel divides in FP32 (correctly rounded), then rounds to e4m3
    q = (x / s[:, None]).astype(np.float32).astype(np.float64)
    assert np.array_equal(oracle.decode_e4m3(got), oracle.decode_e4m3(oracle.encode_e4m3(q)))

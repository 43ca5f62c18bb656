"""The input generators' bfloat16 quantisation: round to nearest, ties to
even, bit for bit as torch converts float32 to bfloat16 (both sides of the
bfloat16 parity tests quantise the same images)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.uniform(0, 1, 50000), 1e3 * rng.standard_normal(50000),
                        [0.0, -0.0, 1.0, 0.5, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9,
                         3 * 2 ** -9 + 1]]).astype(np.float32)
    b = synth.bf16_bits(a)
    t = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(b, t)
    assert np.array_equal(synth.bf16_to_f32(b), torch.from_numpy(a).to(torch.bfloat16).float().numpy())


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between bfloat16 neighbours 1 and 1 + 2^-7: the even one is 1
    assert synth.bf16_to_f32(synth.bf16_bits(np.float32([1 + 2 ** -8])))[0] == 1.0
    assert synth.bf16_to_f32(synth.bf16_bits(np.float32([1 + 3 * 2 ** -8])))[0] == 1 + 2 ** -6

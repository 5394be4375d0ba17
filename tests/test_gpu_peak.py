"""Measured matrix-core rate of each product mode's instruction: within the
published MI355X dense peak, and not far below it."""

import pytest

from paper_1304_2272_amd import binding

pytestmark = pytest.mark.gpu

PUBLISHED = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "int8": 5.0e15}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "int8"])
def test_peak_probe_near_published(precision):
    rate = binding.peak_probe(precision, iters=50000)
    frac = rate / PUBLISHED[precision]
    print(f"{precision}: {rate / 1e12:.1f} T op/s = {frac:.3f} of published", flush=True)
    assert 0.8 < frac < 1.05

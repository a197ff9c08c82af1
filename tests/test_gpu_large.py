"""Large-N parity: the 4096-element streaming array on a 256 x 256 grid
against the FP64 oracle, on the banded two-pass path (the default at this
size) and on the fused path forced to sixteen 64 x 64 sub-transforms; the
self terms come from the separate pass either way."""
import pytest

import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sub", [None, 64], ids=["banded", "fused64"])
def test_stream_array_top_channel_matches_oracle(sub):
    full = synth.workload("stream")
    chans = [63]
    _say(f"case stream array: 4096 elements, 256^2, channel 63, 3 samples, sub {sub}")
    wl = full.subset(chans).with_time(3)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(3), pos, chans=chans)
    got = _run(wl, pos, volt, sub_n=None if sub is None else [sub])
    ref = oracle_images(volt, pos, wl, range(1))
    _check(got, ref, f"stream-{sub}")

"""Large-N parity: the 4096-element streaming array on a 256 x 256 grid
(sixteen 64 x 64 sub-transforms per channel, self terms from the separate
pass) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say

pytestmark = pytest.mark.gpu


def test_stream_array_top_channel_matches_oracle():
    full = synth.workload("stream")
    chans = [63]
    _say("case stream array: 4096 elements, 256^2, channel 63, 3 samples")
    wl = full.subset(chans).with_time(3)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(3), pos, chans=chans)
    got = _run(wl, pos, volt)
    ref = oracle_images(volt, pos, wl, range(1))
    _check(got, ref, "stream")

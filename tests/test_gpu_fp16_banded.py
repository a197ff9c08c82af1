"""FP16 four-step MFMA transform on 256 x 256 channels (precision
EPIC_F16_MFMA, banded path): the 4096-element streaming array and a small
array on a 256^2 grid, a dense 4096-element array (about 30 taps per
cell), 4- and 8-bit voltages, several calls, against the
FP64 oracle to the stated FP16 four-step bound."""
import dataclasses
import json
import os

import numpy as np
import pytest

import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say

pytestmark = pytest.mark.gpu

TOL = json.load(open(os.path.join(os.path.dirname(__file__), "tolerances.json")))["fp16_fourstep"]


def test_stream_array_fp16_fourstep_matches_oracle():
    full = synth.workload("stream")
    chans = [63]
    _say("case fp16 four-step: stream array, 4096 elements, 256^2, channel 63, 3 samples")
    wl = full.subset(chans).with_time(3)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(3), pos, chans=chans)
    got = _run(wl, pos, volt, precision=1)
    _check(got, oracle_images(volt, pos, wl, range(1)), "fp16-4step-stream", TOL["max"],
           TOL["rms"])


@pytest.mark.parametrize("bits", [4, 8])
def test_small_array_256_grid_fp16_fourstep_in_calls(bits):
    wl = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([256]), n_time=24,
                             volt_bits=bits)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case fp16 four-step: 16 elements on 256^2, {bits}-bit, 24 samples in 3 calls")
    ref = oracle_images(volt, pos, wl, [0])
    _check(_run(wl, pos, volt, precision=1, chunks=3), ref, f"fp16-4step-{bits}bit",
           TOL["max"], TOL["rms"])


def test_fp16_fourstep_rounds_alternate_scratch_halves(monkeypatch):
    # 300 samples on a 256^2 grid in rounds of at most 256 (the
    # EPIC_BAND_ROUND cap): two rounds of the banded path (150 + 150
    # samples), the second in the other half of the FP16 scratch
    monkeypatch.setenv("EPIC_BAND_ROUND", "256")
    wl = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([256]), n_time=300)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say("case fp16 four-step: 16 elements on 256^2, 300 samples in one call (two rounds)")
    _check(_run(wl, pos, volt, precision=1), oracle_images(volt, pos, wl, [0]),
           "fp16-4step-rounds", TOL["max"], TOL["rms"])


@pytest.mark.parametrize("n_ant,n_pol", [(15, 2), (16, 1)])
def test_fp16_fourstep_odd_element_count_and_single_feed(n_ant, n_pol):
    # an element count whose voltage blocks are not a multiple of 16 bytes,
    # and one feed (k_band_rows_mf<1> / k_band_cols_mf<1>)
    wl = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([256]), n_time=12,
                             n_ant=n_ant, n_pol=n_pol)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case fp16 four-step: {n_ant} elements x {n_pol} feeds on 256^2, 12 samples in 2 calls")
    _check(_run(wl, pos, volt, precision=1, chunks=2), oracle_images(volt, pos, wl, [0]),
           f"fp16-4step-{n_ant}x{n_pol}", TOL["max"], TOL["rms"])


def test_dense_array_fp16_fourstep_many_taps_per_cell():
    # the streaming array's 4096 elements packed into a 60 m disc: about 30
    # taps per gridded cell, so the half-pair cell sums of the row pass take
    # many roundings, and bands hold far more elements and longer lane lists
    # than on the 300 m disc
    full = dataclasses.replace(synth.workload("stream"), disc_diameter_m=60.0,
                               min_spacing_m=0.5, seed=1093)
    chans = [0, 63]
    _say("case fp16 four-step: 4096 elements in a 60 m disc, 256^2, channels 0 and 63, "
         "4 samples")
    wl = full.subset(chans).with_time(4)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(4), pos, chans=chans)
    got = _run(wl, pos, volt, precision=1)
    _check(got, oracle_images(volt, pos, wl, range(2)), "fp16-4step-dense", TOL["max"],
           TOL["rms"])

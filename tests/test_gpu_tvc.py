"""Parity of the HIP contraction (tvc_contract through the C ABI) with the
float64 oracle, for every mode, several orders and shapes that span many
tiles with ragged tails, and every storage format."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import quant as Q
from oracle import tvc as O
from paper_2501_03121_amd import synth
from _util import TOL, assert_elementwise, host, stored_tensor, vec

pytestmark = pytest.mark.gpu

FMTS = ["f64", "f32", "f16", "bf16", "e4m3"]
SHAPES = [
    (1000003,),            # one long row: split across workgroups
    (33, 1029),            # rows not a multiple of 16 bytes
    (64, 64, 64),
    (7, 13, 5),
    (3, 1, 4, 9),
    (31, 33, 35),
    (128, 96, 80),
    (2, 3, 4, 5, 6, 7),
    (17, 19, 23, 3),
    (8, 4096, 2),          # many rows of a narrow slab
    (3, 50000, 4),         # few slabs, long contracted extent
    (5, 2, 70001),         # few wide rows
    (2, 16, 16, 16, 2, 16),
]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_parity_all_modes(dev, fmt, dims):
    A, S, exact = stored_tensor(dims, fmt, 1, dev)
    for k in range(len(dims)):
        x, xh = vec(dims[k], 10 + k, fmt, dev)
        y = tvc.contract(A, x, k, scale=S)
        torch.cuda.synchronize()
        ref = O.tvc(exact, xh, k)
        err = O.rel_err(host(y), ref)
        assert y.shape == ref.shape
        assert err <= TOL[fmt], (fmt, dims, k, err)
        # and every output on its own
        assert_elementwise(host(y), ref, O.tvc(np.abs(exact), np.abs(xh), k), dims[k], fmt,
                           (dims, k))


@pytest.mark.parametrize("fmt", ["f64", "f32", "f16", "bf16"])
def test_integer_inputs_bitwise(dev, fmt):
    dims = (9, 40, 33, 5)
    base = synth.integers(dims, 3, -8, 8)
    dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[fmt]
    A = torch.from_numpy(base).to(dt).to(dev)
    acc = torch.float64 if fmt == "f64" else torch.float32
    for k, n in enumerate(dims):
        xh = synth.integers(n, 4 + k, -4, 4)
        y = tvc.contract(A, torch.from_numpy(xh).to(acc).to(dev), k)
        assert np.array_equal(host(y), O.tvc(base, xh, k)), (fmt, k)


def test_e4m3_integer_codes_bitwise(dev):
    dims = (6, 20, 17)
    base = synth.integers(dims, 5, -16, 16)
    from oracle import quant as Q
    codes = Q.e4m3_from_f32(base.astype(np.float32))
    A = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(dev)
    S = torch.ones(dims[0], dtype=torch.float32, device=dev)
    for k, n in enumerate(dims):
        xh = synth.integers(n, 6 + k, -3, 3)
        y = tvc.contract(A, torch.from_numpy(xh).float().to(dev), k, scale=S)
        assert np.array_equal(host(y), O.tvc(base, xh, k))


def test_one_hot_is_slice(dev):
    dims = (5, 130, 7, 9)
    A, _, exact = stored_tensor(dims, "f32", 7, dev)
    for k, n in enumerate(dims):
        for m in (0, n // 2, n - 1):
            e = torch.zeros(n, dtype=torch.float32, device=dev)
            e[m] = 1.0
            y = tvc.contract(A, e, k)
            assert np.array_equal(host(y), np.take(exact, m, axis=k))


def test_alpha_beta_and_nan_safety(dev):
    dims = (12, 300, 11)
    A, _, exact = stored_tensor(dims, "f64", 8, dev)
    for k, n in enumerate(dims):
        x, xh = vec(n, 20 + k, "f64", dev)
        odims = O.output_dims(dims, k)
        out = torch.full(odims, float("nan"), dtype=torch.float64, device=dev)
        tvc.contract(A, x, k, alpha=2.5, beta=0.0, out=out)
        assert torch.isfinite(out).all()
        assert O.rel_err(host(out), 2.5 * O.tvc(exact, xh, k)) < 1e-12
        y0 = synth.uniform(odims, 30 + k)
        out = torch.from_numpy(y0).to(dev)
        tvc.contract(A, x, k, alpha=-0.75, beta=1.5, out=out)
        assert O.rel_err(host(out), O.tvc(exact, xh, k, alpha=-0.75, beta=1.5, y=y0)) < 1e-12


@pytest.mark.parametrize("dims", [(1000003,), (3, 50000, 4), (256, 256, 256)])
def test_bitwise_deterministic(dev, dims):
    A, _, _ = stored_tensor(dims, "f32", 9, dev)
    for k, n in enumerate(dims):
        x, _ = vec(n, 40, "f32", dev)
        a = tvc.contract(A, x, k).clone()
        b = tvc.contract(A, x, k)
        assert torch.equal(a, b)


# Contiguous rows that start on a 4-byte boundary but are not whole 16-byte
# vectors: the vector path with a ragged row end, in every family and with
# split contracted extents.  Lengths per format keep rows dword-aligned.
EPV = {"f64": 2, "f32": 4, "f16": 8, "bf16": 8, "e4m3": 16}
RAGGED_LEN = {"f64": (1001, 13, 200001), "f32": (1001, 13, 200001), "f16": (1002, 14, 200002),
              "bf16": (1002, 14, 200002), "e4m3": (1004, 20, 200004)}


def _ragged_cases(fmt):
    lg, sh, huge = RAGGED_LEN[fmt]
    return [
        ((37, lg), 1, "row"),           # long rows
        ((37, lg), 0, "col"),           # column streaming
        ((3000, lg), 0, "col"),         # column streaming, split contracted extent
        ((300, sh), 1, "row"),          # short rows, several per wave
        ((300, sh), 0, "slab"),         # one slab
        ((50, 60, sh), 1, "slab"),      # many slabs
        ((3, 5000, sh), 1, "slab"),     # few slabs, split contracted extent
        ((huge,), 0, "row"),            # one long row split across workgroups
        ((2, 3, lg), 2, "row"),
    ]


@pytest.fixture
def no_stage():
    # the small-slab shapes below would go to the LDS-staged family; turn it
    # off so the row and slab kernels' ragged paths are the ones tested
    from paper_2501_03121_amd import tune
    tune.set_tuning("stage", -1)
    yield
    tune.set_tuning("stage", 0)


@pytest.mark.parametrize("fmt", FMTS)
def test_ragged_vector_rows(dev, fmt, no_stage):
    for dims, k, family in _ragged_cases(fmt):
        A, S, exact = stored_tensor(dims, fmt, 13, dev)
        p = tvc.contract_plan(A, k, scale=S)
        contiguous = int(np.prod(dims[k + 1:])) if k + 1 < len(dims) else dims[k]
        assert p["family"] == family and p["vec"], (fmt, dims, k, p)
        assert p["tail"] == contiguous % EPV[fmt] and p["tail"] > 0, (fmt, dims, k, p)
        x, xh = vec(dims[k], 70 + k, fmt, dev)
        for alpha, beta in ((1.0, 0.0), (0.5, -2.0)):
            y0 = torch.from_numpy(synth.uniform(O.output_dims(dims, k), 80 + k))
            y0 = y0.to(torch.float64 if fmt == "f64" else torch.float32)
            out = y0.to(dev)
            tvc.contract(A, x, k, alpha=alpha, beta=beta, out=out, scale=S)
            ref = O.tvc(exact, xh, k, alpha=alpha, beta=beta, y=host(y0))
            err = O.rel_err(host(out), ref)
            assert err <= TOL[fmt], (fmt, dims, k, alpha, beta, err)
            mag = abs(alpha) * O.tvc(np.abs(exact), np.abs(xh), k) + abs(beta) * np.abs(host(y0))
            assert_elementwise(host(out), ref, mag, dims[k], fmt, (dims, k, alpha, beta))


# Rows of 1- and 2-byte formats whose length is not a whole number of dwords
# start on any byte; they still stream in 16-byte units (loaded at any byte
# address), with a ragged end.
UNALIGNED_LEN = {"f16": (1001, 13, 200001), "bf16": (1001, 13, 200001), "e4m3": (1001, 21, 200003)}


@pytest.mark.parametrize("fmt", ["f16", "bf16", "e4m3"])
def test_unaligned_narrow_rows(dev, fmt, no_stage):
    lg, sh, huge = UNALIGNED_LEN[fmt]
    cases = [((37, lg), 1), ((37, lg), 0), ((3000, lg), 0), ((300, sh), 1), ((300, sh), 0),
             ((50, 60, sh), 1), ((3, 5000, sh), 1), ((huge,), 0), ((2, 3, lg), 2), ((5, 7, lg), 1)]
    for dims, k in cases:
        A, S, exact = stored_tensor(dims, fmt, 15, dev)
        p = tvc.contract_plan(A, k, scale=S)
        contiguous = int(np.prod(dims[k + 1:])) if k + 1 < len(dims) else dims[k]
        assert (contiguous * {"f16": 2, "bf16": 2, "e4m3": 1}[fmt]) % 4 != 0
        assert p["vec"], (fmt, dims, k, p)
        x, xh = vec(dims[k], 75 + k, fmt, dev)
        for alpha, beta in ((1.0, 0.0), (0.5, -2.0)):
            y0 = torch.from_numpy(synth.uniform(O.output_dims(dims, k), 85 + k))
            out = y0.to(torch.float32).to(dev)
            tvc.contract(A, x, k, alpha=alpha, beta=beta, out=out, scale=S)
            ref = O.tvc(exact, xh, k, alpha=alpha, beta=beta, y=host(y0.to(torch.float32)))
            err = O.rel_err(host(out), ref)
            assert err <= TOL[fmt], (fmt, dims, k, alpha, beta, err)
            mag = abs(alpha) * O.tvc(np.abs(exact), np.abs(xh), k) + abs(beta) * np.abs(host(y0))
            assert_elementwise(host(out), ref, mag, dims[k], fmt, (dims, k, alpha, beta))


# Small slabs staged through LDS in blocks of whole slabs: rows of 33-64
# 16-byte units, and slabs of at most 4 KB with a ragged, non-power-of-two or
# very narrow right extent.  The cases cover a single partial block, a ragged
# last block, one-element right extents and several blocks per workgroup.
def _staged_cases(fmt):
    # rows of 33-64 units are staged only in float64
    rows = [((3000, 91), 1), ((7, 11, 91), 2)] if fmt == "f64" else []
    # right extents 12 and 20 are whole 16-byte words in float32 and float64:
    # the staged kernel then reads several columns per LDS word
    words = [((64, 9, 12), 1), ((300, 5, 20), 1)] + ([((500, 6, 32), 1)] if fmt == "e4m3" else [])
    # power-of-two rows narrower than one 16-byte vector (8 and 4 bytes)
    words += {"e4m3": [((600, 5, 8), 1), ((700, 3, 4), 1)], "bf16": [((600, 5, 4), 1)],
              "f16": [((600, 5, 4), 1)]}.get(fmt, [])
    # a long contracted extent: the weights take up to a quarter of the LDS
    # staging buffer, which then holds fewer slabs per block
    big_m = {"f64": 150, "f32": 300, "f16": 600, "bf16": 600, "e4m3": 1300}[fmt]
    return rows + words + [((13,) * 5, 3), ((50, 37, 13), 1), ((1001, 3, 7), 1), ((9, 15, 31), 1),
                           ((3, 5, 7), 1), ((6, 7, 1, 9), 2), ((2, 3, 4, 5, 6, 7), 4),
                           ((40, big_m, 3), 1)]


@pytest.mark.parametrize("fmt", FMTS)
def test_staged_small_slabs(dev, fmt):
    for dims, k in _staged_cases(fmt):
        A, S, exact = stored_tensor(dims, fmt, 17, dev)
        p = tvc.contract_plan(A, k, scale=S)
        assert p["family"] == "stage", (fmt, dims, k, p)
        x, xh = vec(dims[k], 90 + k, fmt, dev)
        for alpha, beta in ((1.0, 0.0), (-1.5, 0.25)):
            y0 = torch.from_numpy(synth.uniform(O.output_dims(dims, k), 95 + k))
            y0 = y0.to(torch.float64 if fmt == "f64" else torch.float32)
            out = y0.to(dev)
            tvc.contract(A, x, k, alpha=alpha, beta=beta, out=out, scale=S)
            ref = O.tvc(exact, xh, k, alpha=alpha, beta=beta, y=host(y0))
            err = O.rel_err(host(out), ref)
            assert err <= TOL[fmt], (fmt, dims, k, alpha, beta, err)
            mag = abs(alpha) * O.tvc(np.abs(exact), np.abs(xh), k) + abs(beta) * np.abs(host(y0))
            assert_elementwise(host(out), ref, mag, dims[k], fmt, (dims, k, alpha, beta))


def test_staged_equals_unstaged_bitwise_on_integers(dev):
    # exact sums: the staged and the row/slab kernels agree bit for bit
    from paper_2501_03121_amd import tune
    for dims, k in _staged_cases("f32")[:6]:
        base = synth.integers(dims, 21, -8, 8)
        A = torch.from_numpy(base).float().to(dev)
        xh = synth.integers(dims[k], 22, -4, 4)
        x = torch.from_numpy(xh).float().to(dev)
        a = tvc.contract(A, x, k).clone()
        tune.set_tuning("stage", -1)
        try:
            assert tvc.contract_plan(A, k)["family"] != "stage"
            b = tvc.contract(A, x, k)
        finally:
            tune.set_tuning("stage", 0)
        assert torch.equal(a, b)
        assert np.array_equal(host(a), O.tvc(base, xh, k))


def test_weights_at_4_byte_offset(dev):
    dims = (40, 256)
    A, _, exact = stored_tensor(dims, "f32", 11, dev)
    big = torch.zeros(257, dtype=torch.float32, device=dev)
    xh = synth.uniform(256, 12)
    big[1:] = torch.from_numpy(xh).float()
    x = big[1:]          # 4-byte aligned, not 16
    y = tvc.contract(A, x, 1)
    assert O.rel_err(host(y), O.tvc(exact, xh.astype(np.float32), 1)) < 1e-5


# Short columns write y through an LDS window in bursts, a wave per strip of
# columns summing all M rows (for problems with enough strips to give every
# workgroup several rounds).  (8, 3 * 2^22 + e/2) makes every workgroup
# flush its window mid-range and ends rows raggedly; the others have a
# ragged 3-d middle mode and one-strip slabs, with a beta term.  On integer
# inputs (exact sums) the window kernel and the column kernel agree bit for
# bit.
def _window_cases(fmt):
    e = EPV[fmt]
    # rows of 20001 narrow elements load in 16-byte units like the others:
    # more of them give enough strips for the window
    lw = 64 if fmt in ("f32", "f64") else 256
    return [((8, (3 << 22) + e // 2), 0), ((lw, 12, 20001), 1), ((4096, 12, 40 * e + e // 2), 1)]


@pytest.mark.parametrize("fmt", FMTS)
def test_output_window(dev, fmt):
    for i, (dims, k) in enumerate(_window_cases(fmt)):
        A, S, exact = stored_tensor(dims, fmt, 23, dev)
        p = tvc.contract_plan(A, k, scale=S)
        assert p["family"] == "col" and p["window"] and p["nsplit"] == 1, (fmt, dims, k, p)
        x, xh = vec(dims[k], 24 + k, fmt, dev)
        if i == 0:
            # (8, n) in mode 0: sampled outputs against the oracle's
            # definition, one by one
            ah = host(tvc.contract(A, x, k, scale=S))
            xs = xh.astype(np.float64)
            js = np.concatenate([synth.integers(60, 26, 0, dims[1] - 1).astype(np.int64),
                                 np.arange(dims[1] - 4, dims[1])])
            for j in js:
                want = float(np.dot(exact[:, j], xs))
                bound = TOL[fmt] * float(np.abs(exact[:, j]) @ np.abs(xs))
                assert abs(float(ah[j]) - want) <= bound, (fmt, j)
            continue
        y0 = synth.uniform(O.output_dims(dims, k), 25 + k)
        out = torch.from_numpy(y0).to(torch.float64 if fmt == "f64" else torch.float32).to(dev)
        tvc.contract(A, x, k, alpha=0.5, beta=-1.25, out=out, scale=S)
        ref = O.tvc(exact, xh, k, alpha=0.5, beta=-1.25, y=y0)
        assert O.rel_err(host(out), ref) <= TOL[fmt], (fmt, dims, k)


def test_output_window_equals_column_kernel_on_integers(dev):
    from paper_2501_03121_amd import tune
    for dims, k in _window_cases("f32"):
        base = synth.integers(dims, 27, -8, 8)
        A = torch.from_numpy(base).float().to(dev)
        xh = synth.integers(dims[k], 28, -4, 4)
        x = torch.from_numpy(xh).float().to(dev)
        assert tvc.contract_plan(A, k)["window"]
        a = tvc.contract(A, x, k).clone()
        tune.set_tuning("col", 0, -1)
        try:
            assert not tvc.contract_plan(A, k)["window"]
            b = tvc.contract(A, x, k)
        finally:
            tune.reset()
        assert torch.equal(a, b), (dims, k)
        if np.prod(dims) <= 1 << 25:
            assert np.array_equal(host(a), O.tvc(base, xh, k)), (dims, k)


# The slab, short-row and staged kernels with the output window: many short
# rows, many slabs of a power-of-two right extent (the slab family), and
# many ragged small slabs (the LDS-staged family, or the slab family with
# staging off).  They sum in the same order as without the window, so the
# two agree bit for bit on any input.
SLAB_R = {"f64": 16, "f32": 32, "f16": 64, "bf16": 64, "e4m3": 128}


def _windowed_cases(fmt):
    lg, sh, _ = RAGGED_LEN[fmt]
    return [((1200000, sh), 1, "row", False), ((70000, 9, SLAB_R[fmt]), 1, "slab", False),
            ((150000, 9, sh), 1, "slab", True), ((20000, 7, 8, sh), 3, "row", False),
            ((300000, 9, sh), 1, "stage", False)]


@pytest.mark.parametrize("fmt", FMTS)
def test_windowed_rows_and_slabs(dev, fmt):
    from paper_2501_03121_amd import tune
    for dims, k, family, nostage in _windowed_cases(fmt):
        A, S, exact = stored_tensor(dims, fmt, 29, dev)
        if nostage:
            tune.set_tuning("stage", -1)
        try:
            p = tvc.contract_plan(A, k, scale=S)
            # a staged block's outputs must fit half of its window, 8 KB for
            # the narrow formats: their 32 KB blocks of 9 x 14 or 9 x 20 slabs do not
            want_win = family != "stage" or fmt in ("f32", "f64")
            assert p["family"] == family and p["window"] == want_win, (fmt, dims, k, p)
            x, xh = vec(dims[k], 30 + k, fmt, dev)
            y0 = synth.uniform(O.output_dims(dims, k), 31 + k)
            out = torch.from_numpy(y0).to(torch.float64 if fmt == "f64" else torch.float32).to(dev)
            a = tvc.contract(A, x, k, alpha=0.5, beta=-1.25, out=out.clone(), scale=S)
            tune.set_tuning("col", 0, -1)
            assert not tvc.contract_plan(A, k, scale=S)["window"]
            b = tvc.contract(A, x, k, alpha=0.5, beta=-1.25, out=out.clone(), scale=S)
        finally:
            tune.reset()
        assert torch.equal(a, b), (fmt, dims, k)
        ref = O.tvc(exact, xh, k, alpha=0.5, beta=-1.25, y=y0)
        assert O.rel_err(host(a), ref) <= TOL[fmt], (fmt, dims, k)


# Column strips without the window (M above 256): a wave streams all M rows
# of a strip of 64, 128 or 256 column units.  Large enough for every wave to
# get a strip, so the tensors are made on the device and outputs are checked
# one by one against the oracle's definition on sampled columns, the ragged
# last columns included.
def _device_stored(dims, fmt, seed, dev):
    A32 = synth.device_normal(dims, seed, dev)
    if fmt == "f32":
        return A32, None, lambda idx: A32[idx].double().cpu().numpy()
    if fmt == "f64":
        A = A32.double()
        return A, None, lambda idx: A[idx].cpu().numpy()
    A, S = tvc.quantize(A32, fmt)
    if fmt == "e4m3":
        def exact(idx):
            codes = A[idx].view(torch.uint8).cpu().numpy()
            return Q.e4m3_to_f64(codes) * float(S[idx[0]])
        return A, S, exact
    raw = lambda idx: A[idx].view(torch.int16).cpu().numpy().view(np.uint16)
    conv = Q.bf16_to_f64 if fmt == "bf16" else Q.f16_to_f64
    return A, None, lambda idx: conv(raw(idx))


@pytest.mark.parametrize("fmt", FMTS)
def test_column_strips(dev, fmt):
    e = EPV[fmt]
    # strips of 4, 2 and 1 units per lane in float32 (fewer strips as the
    # tensor shrinks); the smaller cases may fall back to the split column
    # kernel in the narrow formats, which must agree all the same
    for i, dims in enumerate([(1, 260, (1 << 20) + e // 2), (4, 260, (1 << 17) + e // 2),
                              (16, 260, (1 << 14) + e // 2)]):
        A, S, exact = _device_stored(dims, fmt, 41, dev)
        p = tvc.contract_plan(A, 1, scale=S)
        assert p["family"] == "col" and not p["window"], (fmt, dims, p)
        assert i > 0 or p["strip_units"] > 0, (fmt, dims, p)
        if fmt == "f32":
            assert p["strip_units"] == (4, 2, 1)[i], (dims, p)
        x, xh = vec(dims[1], 42, fmt, dev)
        yh = host(tvc.contract(A, x, 1, scale=S))
        xs = xh.astype(np.float64)
        g = synth.rng(43)
        cols = np.concatenate([g.integers(0, dims[2], 48), np.arange(dims[2] - 5, dims[2])])
        for l in (0, dims[0] - 1):
            for j in cols:
                a = exact((l, slice(None), int(j)))
                want = float(a @ xs)
                bound = TOL[fmt] * float(np.abs(a) @ np.abs(xs))
                assert abs(float(yh[l, j]) - want) <= bound, (fmt, dims, l, j)


# Column strips with very short contracted extents: the remainder block of
# M mod (rows per batch) rows in every strip shape (4 or 8 waves, 1 to 4
# units per lane), on integer inputs against the plain column kernel and
# the oracle, bit for bit.
@pytest.mark.parametrize("M", [1, 2, 3, 5, 7, 9, 31, 33, 37])
def test_column_strips_short_extents(dev, M):
    from paper_2501_03121_amd import tune
    for R in (1 << 16, 5000 * 4 + 1):
        dims = (64, M, R)
        base = synth.integers(dims, 60 + M, -8, 8)
        A = torch.from_numpy(base).float().to(dev)
        xh = synth.integers(M, 61, -4, 4)
        x = torch.from_numpy(xh).float().to(dev)
        p = tvc.contract_plan(A, 1)
        assert p["family"] == "col" and p["strip_units"] > 0, (dims, p)
        a = tvc.contract(A, x, 1).clone()
        tune.set_tuning("col", 0, -1)
        try:
            b = tvc.contract(A, x, 1)
        finally:
            tune.reset()
        assert torch.equal(a, b), (dims, p)
        assert np.array_equal(host(a), O.tvc(base, xh, 1)), (dims, p)


# Column strips whose rows are 1 MB apart (4 units per lane, output window):
# each workgroup starts at its own row and wraps around, including the
# remainder block of M mod (rows per batch) rows.  On integer inputs the sum
# is exact in any order, so the result equals the plain column kernel's and
# the oracle's bit for bit.
@pytest.mark.parametrize("M", [1, 3, 5, 17])
def test_column_strips_rotated_rows(dev, M):
    from paper_2501_03121_amd import tune
    for fmt, R in (("f32", 1 << 18), ("bf16", 1 << 19)):
        if fmt == "bf16" and M != 3:
            continue
        dims = (32, M, R)
        base = synth.integers(dims, 70 + M, -8, 8)
        dt = torch.float32 if fmt == "f32" else torch.bfloat16
        A = torch.from_numpy(base).to(dt).to(dev)
        xh = synth.integers(M, 71, -4, 4)
        x = torch.from_numpy(xh).float().to(dev)
        p = tvc.contract_plan(A, 1)
        assert p["family"] == "col" and p["window"] and p["strip_units"] == 4, (fmt, dims, p)
        assert p["row_rotation"], (fmt, dims, p)
        a = tvc.contract(A, x, 1).clone()
        tune.set_tuning("col", 0, -1)
        try:
            assert not tvc.contract_plan(A, 1)["row_rotation"]
            b = tvc.contract(A, x, 1)
        finally:
            tune.reset()
        assert torch.equal(a, b), (fmt, dims)
        assert np.array_equal(host(a), O.tvc(base, xh, 1)), (fmt, dims)


# E4M3 rows that are one pass of a wave (1024 and 3072 bytes: 8 and 2 rows
# per wave) take a path that loads the next row group before summing the
# current one; odd row counts end inside a group.  Parity with the oracle,
# with an alpha/beta epilogue.
def test_e4m3_one_pass_rows(dev):
    for dims in ((301, 1024), (37, 3072), (5, 7, 1024)):
        k = len(dims) - 1
        A, S, exact = stored_tensor(dims, "e4m3", 80, dev)
        p = tvc.contract_plan(A, k, scale=S)
        assert p["family"] == "row" and p["nsplit"] == 1 and p["tail"] == 0, (dims, p)
        x, xh = vec(dims[k], 81, "e4m3", dev)
        y0 = synth.uniform(O.output_dims(dims, k), 82)
        out = torch.from_numpy(y0).float().to(dev)
        tvc.contract(A, x, k, alpha=0.75, beta=-0.5, out=out, scale=S)
        ref = O.tvc(exact, xh, k, alpha=0.75, beta=-0.5, y=y0)
        assert O.rel_err(host(out), ref) <= TOL["e4m3"], dims

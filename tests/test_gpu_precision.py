"""Error of every narrow-storage result against the float64 oracle on the
original float32 data, at the full 1024^3 and 32^6 sizes (sampled outputs),
for the contraction in every mode and for the HOPM eigenvalue.

The measured errors are printed; the assertions are the bounds the formats
allow: bf16 and E4M3 round to 8 and 4 significant bits, fp16 to 11.
"""
import json

import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import hopm as H
from oracle import tvc as O
from paper_2501_03121_amd import synth
from _util import host

pytestmark = pytest.mark.gpu

SHAPES = [(1024, 1024, 1024), (32, 32, 32, 32, 32, 32)]
# norm-wise relative error bounds of a contraction whose inputs were rounded
# to the format (random-sign rounding errors average out, so well below the
# per-element unit roundoff)
BOUND = {"f32": 1e-5, "bf16": 4e-3, "f16": 5e-4, "e4m3": 6e-2}


@pytest.mark.parametrize("dims", SHAPES, ids=["1024^3", "32^6"])
def test_narrow_storage_tvc_error(dev, dims):
    A = synth.device_normal(dims, 100, dev)
    Ah = A.cpu().numpy()
    errs = {}
    stored = {"f32": (A, None)}
    for fmt in ("bf16", "f16", "e4m3"):
        stored[fmt] = tvc.quantize(A, fmt)
    for k in range(len(dims)):
        xh = synth.unit_vectors([dims[k]], 300 + k)[0].astype(np.float32)
        x = torch.from_numpy(xh).to(dev)
        u, _, v = O.matricized_dims(dims, k)
        g = synth.rng(7 + k)
        lr = np.stack([g.integers(0, u, 2048), g.integers(0, v, 2048)], axis=1)
        ref = O.tvc_sample(Ah, xh, k, lr)
        for fmt, (Aq, S) in stored.items():
            y = host(tvc.contract(Aq, x, k, scale=S)).reshape(u, v)[lr[:, 0], lr[:, 1]]
            e = O.rel_err(y, ref)
            errs[f"{fmt}_mode{k}"] = e
            assert e < BOUND[fmt], (fmt, k, e)
    print(json.dumps({"x".join(map(str, dims)): errs}))


@pytest.mark.timeout(900)
def test_narrow_storage_lambda_error(dev):
    # 32^6 planted tensor, warm start: lambda of every storage format (with
    # and without float32 refinement to the same tol) against the float64 solve
    dims = SHAPES[1]
    A, a = synth.device_planted(dims, 10.0, 0.1, 200, dev)
    x0 = synth.warm_start(a, 0.9, 400)
    ref = H.hopm(A.cpu().numpy(), x0, tol=1e-9, max_sweeps=60)
    out = {"oracle_lambda": ref.lam, "oracle_sweeps": ref.sweeps}
    for fmt in ("f32", "bf16", "f16", "e4m3"):
        Aq, S = (A, None) if fmt == "f32" else tvc.quantize(A, fmt)
        for refine in (0, 1):
            if fmt == "f32" and refine:
                continue
            x = tvc.pack_vectors(x0, dev)
            r = tvc.hopm_solve(Aq, x, tol=1e-6, max_sweeps=200, scale=S,
                               A_refine=A if refine else None, refine_sweeps=60 if refine else 0)
            e = abs(r.lam - ref.lam) / ref.lam
            out[f"{fmt}{'+refine' if refine else ''}"] = {"lambda_rel_err": e, "sweeps": r.sweeps,
                                                        "refine_sweeps": r.refine_sweeps}
            assert r.status == 0 and r.delta < 1e-6
            bound = 1e-5 if fmt == "f32" or refine else (3e-3 if fmt == "e4m3" else 1e-3)
            assert e <= bound, (fmt, refine, e)
    print(json.dumps(out))

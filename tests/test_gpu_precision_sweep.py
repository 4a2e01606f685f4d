"""Precision sweep: textures of the small workload (4 x 256^2, 9 levels,
bounded blocks, modes uniform over 14), MLP 12-64-64-10, 2^24 uniform
queries, the MLP in fp32 (vector ALU), fp32 / bf16 / fp16 / fp8 on MFMA with
fp32 accumulation. Reports per-channel max and mean absolute error against the
fp64 oracle over every query; the report is also written, as JSON, to the
path in the environment variable BCF_PRECISION_SWEEP_JSON when it is set."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BARS = {"FP32": 1e-5, "FP32_MFMA": 1e-5, "FP16": 2e-3, "BF16": 2e-2, "FP8": None}


def test_precision_sweep():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_16121_amd as bcf
    wl = synth.WORKLOADS["sweep"]
    m = synth.workload_material(wl, variant="B")
    q = synth.workload_queries(wl)
    host = oracle.Material.from_synth(m)
    print(f"oracle on {len(q)} queries", flush=True)
    ref = oracle.decode(host, q)
    mat = bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params)
    qd = torch.from_numpy(q).cuda()
    # static fp8 activation scales from a separate calibration batch
    calib = synth.uniform_queries(1 << 16, synth.rng(1234), wl.s_max)
    mat.set_act_absmax(bcf.calibrate(mat, torch.from_numpy(calib).cuda()))
    report = {"workload": "4 x 256^2 BC6H pyramids (9 levels, bounded, modes uniform over 14), "
                          "MLP 12-64-64-10, 2^24 uniform queries", "queries": len(q),
              "output_range": float(np.abs(ref).max()), "precisions": {}}
    for name, bar in BARS.items():
        prec = bcf.Precision[name]
        ws = bcf.prepare(mat, prec)
        out = bcf.decode(mat, ws, qd, prec)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        err = np.abs(got - ref)
        entry = {"max_abs_err": err.max(axis=0).tolist(), "mean_abs_err": err.mean(axis=0).tolist(),
                 "max_abs_err_all": float(err.max()), "mean_abs_err_all": float(err.mean())}
        report["precisions"][name] = entry
        print(f"{name}: max {entry['max_abs_err_all']:.3e} mean {entry['mean_abs_err_all']:.3e}", flush=True)
        assert np.isfinite(got).all()
        if bar is not None:
            assert err.max() <= bar
        del ws, out
    path = os.environ.get("BCF_PRECISION_SWEEP_JSON")
    if path:
        with open(path, "w") as f:
            json.dump(report, f, indent=1)

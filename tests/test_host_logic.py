"""Host-side logic of the library checked on the CPU (no GPU needed): the
judge's offsets and weights and the network's inputs that demag_quad_predict
computes in C++ equal, bit for bit, the recipe written in Python
(inputs.fit_offsets, inputs.quad_features) that the tests and the training
cases use; and the benchmark's writer of the HBM counter summary."""
import numpy as np

from paper_1212_3509_amd import api, inputs


def _grids():
    rng = np.random.default_rng(17)
    grids = [tuple(int(v) for v in rng.integers(1, 300, 3)) for _ in range(150)]
    grids += [tuple(int(v) for v in rng.integers(32, 65, 3)) for _ in range(150)]
    grids += [(1, 1, 1), (2, 1, 3), (4, 4, 4), (5, 5, 5), (128, 128, 128), (256, 256, 256), (256, 256, 4),
              (1024, 1024, 1024), (4096, 4096, 4096), (4096, 7, 300), (33, 4096, 1)]
    return grids


def test_library_offsets_equal_the_python_recipe():
    for n in _grids():
        J, w = api.quad_offsets(n)
        Jp, wp = inputs.fit_offsets(n)
        assert np.array_equal(J, Jp), n
        assert np.array_equal(w, wp), n


def test_library_features_equal_the_python_recipe():
    rng = np.random.default_rng(5)
    for n in _grids()[:200]:
        h = 1.0 / max(n)
        tol = float(rng.uniform(-9, -4))
        R = int(rng.integers(16, 33))
        x = api.quad_features(n, h, tol, R)
        xp = inputs.quad_features([n], [h], [tol], [R])[0]
        assert np.array_equal(x.view(np.uint32), xp.view(np.uint32)), (n, tol, R)


def test_traffic_summary_writer(tmp_path, monkeypatch):
    """bench.py --write-traffic: per-stage medians of FETCH_SIZE / WRITE_SIZE
    scaled by what the counters read for the calibration copy, the copy
    found among the elementwise kernels as the one that also reads."""
    import csv
    import json

    import bench
    src = tmp_path / "traffic.json"
    src.write_text(json.dumps({"workload": "w", "kernels": {
        "fp64/z/nout2": {"kernel": "k_left<double, 8, 2, 2, true>"}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(src))
    mib = 4
    fill = "void at::native::vectorized_elementwise_kernel<4, FillFunctor<float>>(int)"
    copy = "void at::native::vectorized_elementwise_kernel<4, MulFunctor<float>>(int)"
    stage = "void demag::(anonymous namespace)::k_left<double, 8, 2, 2, true>(demag::MPJob const*)"

    def write(path, counter, rows):
        with open(path, "w", newline="") as fh:
            wr = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            wr.writeheader()
            for k, v in rows:
                wr.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})
    kib = mib * 1024
    write(tmp_path / "f.csv", "FETCH_SIZE", [(fill, 0.0), (copy, kib / 2), (stage, 100.0), (stage, 300.0),
                                            (stage, 200.0)])
    write(tmp_path / "w.csv", "WRITE_SIZE", [(fill, kib), (copy, kib), (stage, 50.0)])
    bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), mib)
    rec = json.loads(src.read_text())
    cal = rec["copy_calibration"]
    assert cal["fetch_scale"] == 2.0 and cal["write_scale"] == 1.0
    k = rec["kernels"]["fp64/z/nout2"]
    assert k["fetch_kib"] == 200.0 and k["write_kib"] == 50.0
    assert k["hbm_bytes_per_launch"] == 1024 * (200.0 * 2.0 + 50.0)
    assert rec["kernel_source_sha256"] == bench._kernel_source_hash()

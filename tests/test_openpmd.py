"""openPMD-shaped output: a small box written and read back (host tensors;
the writer only moves data), every attribute the openPMD 1.1.0 base
standard requires is present, and the data round-trip exactly (the split
position form reassembled as cell + offset)."""
import numpy as np

import pic_inputs as pi
from paper_2303_12873_amd import openpmd


def test_write_read_round_trip(tmp_path):
    wl = pi.uniform_box((6, 5, 4), 2, 0.05, 0.1, 2, 9900, "cpu", tile=(4, 4, 4),
                        fields="fourier", species=("e", "i"))
    box = wl.boxes[0]
    J = np.random.default_rng(1).normal(size=(3, box.ncells))
    e, i = wl.species
    fn = openpmd.write_iteration(
        str(tmp_path), 7, 7 * box.dt, box, {"E": wl.E[0], "B": wl.B[0], "J": J},
        {"electrons": {"q": e.q, "m": e.m, "x": e.x, "u": e.u, "w": e.w},
         "ions": {"q": i.q, "m": i.m, "x": None, "cell": i.cell, "off": i.off, "u": i.u,
                  "w": i.w}})
    doc = openpmd.read_iteration(fn)
    assert openpmd.check_standard(doc) == []
    it = doc["data"]["7"]
    assert abs(it["attributes"]["time"] - 7 * box.dt) < 1e-15
    ex = np.array(it["meshes"]["E"]["x"]["data"]).reshape(-1)
    np.testing.assert_array_equal(ex, wl.E[0][0].numpy())
    assert it["meshes"]["E"]["x"]["attributes"]["position"] == [0.0, 0.0, 0.5]   # (z, y, x)
    assert it["meshes"]["B"]["x"]["attributes"]["position"] == [0.5, 0.5, 0.0]
    np.testing.assert_array_equal(np.array(it["meshes"]["J"]["z"]["data"]).reshape(-1), J[2])
    pe = it["particles"]["electrons"]
    np.testing.assert_array_equal(np.array(pe["position"]["x"]["data"]), e.x[0].numpy())
    np.testing.assert_array_equal(np.array(pe["weighting"]["data"]), e.w.numpy())
    pz = np.array(it["particles"]["ions"]["position"]["z"]["data"])
    np.testing.assert_array_equal(pz, i.x[2].numpy())         # split form reassembled exactly
    mom = np.array(it["particles"]["ions"]["momentum"]["y"]["data"])
    np.testing.assert_allclose(mom, i.u[1].numpy() * i.m, rtol=1e-15)


def test_missing_attribute_is_reported(tmp_path):
    wl = pi.uniform_box((4, 4, 4), 1, 0.05, 0.1, 1, 9901, "cpu", tile=(4, 4, 4))
    box = wl.boxes[0]
    fn = openpmd.write_iteration(str(tmp_path), 0, 0.0, box, {"E": wl.E[0]}, {})
    doc = openpmd.read_iteration(fn)
    del doc["data"]["0"]["meshes"]["E"]["attributes"]["gridSpacing"]
    del doc["attributes"]["basePath"]
    assert sorted(openpmd.check_standard(doc)) == ["/basePath", "meshes/E/gridSpacing"]

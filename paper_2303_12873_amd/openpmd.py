"""openPMD-shaped output of the PIC state (fields and particles of one box).

The paper's codes write their data in the openPMD standard (Sec. IV); this
writer produces one iteration per file in the layout of openPMD 1.1.0 with
the JSON encoding of the openPMD-api's JSON backend: a tree of groups whose
"attributes" hold the standard's attributes and whose datasets hold
``{"datatype": ..., "extent": [...], "data": nested lists}``.  Only the
output layer lives here (device arrays are copied to the host and
rearranged); no arithmetic of the method.

Conventions written into the attributes: normalised units (c = eps0 = mu0 =
1, lengths in cells): unitSI = 1 and gridUnitSI = 1 flag them as
dimensionless.  Field components carry their Yee stagger in ``position``
(in cell units, x fastest: E_x at (1/2, 0, 0) ...).  Particle positions are
the cell-unit coordinates of the box (the split form is reassembled as
cell + offset in FP64), positionOffset is zero, momentum is u = gamma v
per unit mass times the species mass.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional

import numpy as np

OPENPMD_VERSION = "1.1.0"

# unitDimension exponents (L, M, T, I, theta, N, J) of the SI base units
_DIM = {
    "E": [1, 1, -3, -1, 0, 0, 0],
    "B": [0, 1, -2, -1, 0, 0, 0],
    "J": [-2, 0, 0, 1, 0, 0, 0],
    "position": [1, 0, 0, 0, 0, 0, 0],
    "momentum": [1, 1, -1, 0, 0, 0, 0],
    "weighting": [0, 0, 0, 0, 0, 0, 0],
    "charge": [0, 0, 1, 1, 0, 0, 0],
    "mass": [0, 1, 0, 0, 0, 0, 0],
}


def _dataset(a: np.ndarray) -> dict:
    a = np.asarray(a)
    dt = {np.dtype(np.float64): "DOUBLE", np.dtype(np.float32): "FLOAT",
          np.dtype(np.int32): "INT", np.dtype(np.int64): "LONG"}[a.dtype]
    return {"datatype": dt, "extent": list(a.shape), "data": a.tolist()}


def _stagger(name: str, comp: int) -> List[float]:
    """Yee position of component comp (0 x, 1 y, 2 z), listed (x, y, z)."""
    pos = [0.0, 0.0, 0.0]
    for d in range(3):
        on = (d == comp) if name in ("E", "J") else (d != comp)
        pos[d] = 0.5 if on else 0.0
    return pos


def _to_host(t) -> np.ndarray:
    try:
        import torch
        if isinstance(t, torch.Tensor):
            return t.detach().cpu().numpy()
    except ImportError:
        pass
    return np.asarray(t)


def write_iteration(path: str, iteration: int, time: float, box, fields: Dict[str, object],
                    species: Dict[str, dict], cell_base: int = 0) -> str:
    """Writes ``path/openpmd_<iteration>.json``.

    box: a box description (dim, n, dx, dt).  fields: {"E": (3, total cells)
    array, "B": ..., "J": ...} (any of them; host or device tensors; the box
    occupies cells [cell_base, cell_base + ncells)).  species: {name:
    {"q": q, "m": m, "x": (3, np) positions or None, "cell": (np,) and
    "off": (3, np) for the split form, "u": (3, np), "w": (np,)}}.
    Returns the file name."""
    n = [int(v) for v in box.n]
    nc = n[0] * n[1] * n[2]
    axis = ["x", "y", "z"]
    meshes = {}
    for name, arr in fields.items():
        a = _to_host(arr)[:, cell_base:cell_base + nc]
        comps = {}
        for c in range(3):
            d = _dataset(a[c].reshape(n[2], n[1], n[0]))
            comps[axis[c]] = {"attributes": {"unitSI": 1.0,
                                             "position": _stagger(name, c)[::-1]},
                              **d}
        meshes[name] = {
            "attributes": {
                "geometry": "cartesian", "dataOrder": "C",
                "axisLabels": ["z", "y", "x"],
                "gridSpacing": [float(box.dx[2]), float(box.dx[1]), float(box.dx[0])],
                "gridGlobalOffset": [0.0, 0.0, 0.0], "gridUnitSI": 1.0,
                "unitDimension": _DIM[name], "timeOffset": 0.0,
            },
            **comps,
        }
    parts = {}
    for name, sp in species.items():
        u = _to_host(sp["u"]).astype(np.float64)
        w = _to_host(sp["w"]).astype(np.float64)
        npart = int(w.shape[0])
        if sp.get("x") is not None:
            x = _to_host(sp["x"]).astype(np.float64)
        else:
            cell = _to_host(sp["cell"]).astype(np.int64)
            off = _to_host(sp["off"]).astype(np.float64)
            x = np.stack([cell % n[0] + off[0], (cell // n[0]) % n[1] + off[1],
                          cell // (n[0] * n[1]) + off[2]])
        rec = {
            "position": {"attributes": {"unitDimension": _DIM["position"], "timeOffset": 0.0}},
            "positionOffset": {"attributes": {"unitDimension": _DIM["position"],
                                              "timeOffset": 0.0}},
            "momentum": {"attributes": {"unitDimension": _DIM["momentum"], "timeOffset": 0.0}},
            "weighting": {"attributes": {"unitDimension": _DIM["weighting"], "timeOffset": 0.0,
                                         "unitSI": 1.0, "macroWeighted": 1,
                                         "weightingPower": 1.0}, **_dataset(w)},
            "charge": {"attributes": {"unitDimension": _DIM["charge"], "timeOffset": 0.0,
                                      "unitSI": 1.0, "value": float(sp["q"]),
                                      "shape": [npart], "macroWeighted": 0,
                                      "weightingPower": 1.0}},
            "mass": {"attributes": {"unitDimension": _DIM["mass"], "timeOffset": 0.0,
                                    "unitSI": 1.0, "value": float(sp["m"]), "shape": [npart],
                                    "macroWeighted": 0, "weightingPower": 1.0}},
        }
        for d in range(3):
            rec["position"][axis[d]] = {"attributes": {"unitSI": 1.0}, **_dataset(x[d])}
            rec["positionOffset"][axis[d]] = {"attributes": {"unitSI": 1.0, "value": 0.0,
                                                             "shape": [npart]}}
            rec["momentum"][axis[d]] = {"attributes": {"unitSI": 1.0},
                                        **_dataset(u[d] * float(sp["m"]))}
        for k in ("position", "positionOffset", "momentum"):
            rec[k]["attributes"].update({"macroWeighted": 0, "weightingPower": 1.0})
        parts[name] = rec
    doc = {
        "attributes": {
            "openPMD": OPENPMD_VERSION, "openPMDextension": 0, "basePath": "/data/%T/",
            "meshesPath": "meshes/", "particlesPath": "particles/",
            "iterationEncoding": "fileBased", "iterationFormat": "openpmd_%T.json",
            "software": "paper_2303_12873_amd", "date": "",
        },
        "data": {
            str(int(iteration)): {
                "attributes": {"time": float(time), "dt": float(box.dt), "timeUnitSI": 1.0},
                "meshes": meshes,
                "particles": parts,
            }
        },
    }
    os.makedirs(path, exist_ok=True)
    fn = os.path.join(path, f"openpmd_{int(iteration)}.json")
    with open(fn, "w") as f:
        json.dump(doc, f)
    return fn


def read_iteration(fn: str) -> dict:
    """The JSON tree written by write_iteration."""
    with open(fn) as f:
        return json.load(f)


REQUIRED_ROOT = ("openPMD", "openPMDextension", "basePath", "meshesPath", "particlesPath",
                 "iterationEncoding", "iterationFormat")
REQUIRED_ITERATION = ("time", "dt", "timeUnitSI")
REQUIRED_MESH = ("geometry", "dataOrder", "axisLabels", "gridSpacing", "gridGlobalOffset",
                 "gridUnitSI", "unitDimension", "timeOffset")
REQUIRED_RECORD = ("unitDimension", "timeOffset")


def check_standard(doc: dict) -> List[str]:
    """Names of required openPMD 1.1.0 attributes missing from a tree."""
    missing = [f"/{a}" for a in REQUIRED_ROOT if a not in doc["attributes"]]
    for it, g in doc["data"].items():
        missing += [f"/data/{it}/{a}" for a in REQUIRED_ITERATION if a not in g["attributes"]]
        for m, rec in g.get("meshes", {}).items():
            missing += [f"meshes/{m}/{a}" for a in REQUIRED_MESH if a not in rec["attributes"]]
            for c, comp in rec.items():
                if c != "attributes" and "unitSI" not in comp["attributes"]:
                    missing.append(f"meshes/{m}/{c}/unitSI")
        for s, sp in g.get("particles", {}).items():
            for r in ("position", "positionOffset"):
                if r not in sp:
                    missing.append(f"particles/{s}/{r}")
            for r, rec in sp.items():
                missing += [f"particles/{s}/{r}/{a}" for a in REQUIRED_RECORD
                            if a not in rec["attributes"]]
    return missing

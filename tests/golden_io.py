"""Parser for the hand-worked fixtures under tests/golden/ (see the derivation in each file)."""
from __future__ import annotations

import dataclasses
import glob
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NEXT_DIR = os.path.join(GOLDEN_DIR, "next")
METHODS = {"basic": 0, "dense": 1, "sparse": 2, "difference": 3}
TRANSFORMS = {"log": 0, "linear": 1}
THRESH = {"reference": 0, "memoryless": 1}


@dataclasses.dataclass
class Golden:
    name: str
    cfg: Dict[str, object]
    frames: np.ndarray                 # uint8 [T, H, W]
    t_us: List[int]
    flows: Optional[np.ndarray]        # float32 [T-1, H, W, 2] (zeros where absent)
    events: List[List[Tuple[int, int, int, int]]]   # per interval: (t, x, y, p)
    lref: np.ndarray                   # float32 [H, W]


def load(path: str) -> Golden:
    cfg: Dict[str, object] = {}
    frames, ts, flows = [], [], {}
    events: List[List[Tuple[int, int, int, int]]] = []
    lref = None
    for raw in open(path):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        head, _, rest = line.partition(" ")
        if head == "config":
            for kv in rest.split():
                k, v = kv.split("=")
                cfg[k] = v
        elif head == "frame":
            t, _, vals = rest.partition(":")
            ts.append(int(t))
            frames.append([int(v) for v in vals.split()])
        elif head == "flow":
            i, _, vals = rest.partition(":")
            flows[int(i)] = [float(v) for v in vals.split()]
        elif head == "interval":
            assert int(rest) == len(events) + 1
            events.append([])
        elif head == "event":
            t, x, y, p = rest.split()
            events[-1].append((int(t), int(x), int(y), 1 if p == "+" else -1))
        elif head == "lref":
            lref = [float(v) for v in rest.split()]
        else:
            raise ValueError(f"{path}: bad line {raw!r}")
    W, H = int(cfg["width"]), int(cfg["height"])
    out_cfg = dict(method=METHODS[cfg["method"]], transform=TRANSFORMS[cfg["transform"]],
                   c_pos=float(cfg["c_pos"]), c_neg=float(cfg["c_neg"]),
                   n_interp=int(cfg["n_interp"]), mask_threshold=float(cfg["mask"]))
    if "thresh" in cfg:
        out_cfg["thresh_mode"] = THRESH[cfg["thresh"]]
    fr = np.array(frames, dtype=np.uint8).reshape(len(frames), H, W)
    fl = np.zeros((len(frames) - 1, H, W, 2), dtype=np.float32)
    for i, vals in flows.items():
        fl[i - 1] = np.array(vals, dtype=np.float32).reshape(H, W, 2)
    return Golden(os.path.basename(path), out_cfg, fr, ts, fl, events,
                  np.array(lref, dtype=np.float32).reshape(H, W))


def all_fixtures() -> List[str]:
    """Fixtures of the reference-level thresholding of the three frame methods."""
    return sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt")))


def next_fixtures() -> List[str]:
    """Fixtures of the memoryless thresholding and of the difference-frame method."""
    return sorted(glob.glob(os.path.join(NEXT_DIR, "*.txt")))

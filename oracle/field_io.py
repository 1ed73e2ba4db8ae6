"""The oracle's own reader of field files (<prefix>.npz + <prefix>.json).

Independent of the product loader; arrays are read with allow_pickle=False
and the manifest as plain JSON."""
import json

import numpy as np


def load_field(prefix):
    """Reads the field files of this repository (npz + json); no passage of the paper."""
    with open(prefix + ".json") as fh:
        meta = json.load(fh)
    if meta.get("format") != "vrn-field-1":
        raise ValueError("not a vrn-field-1 file")
    with np.load(prefix + ".npz", allow_pickle=False) as z:
        arr = {k: z[k] for k in z.files}
    field = dict(meta)
    for k in ("level_res", "hash_primes", "tables", "occ_bits", "aabb_min"):
        field[k] = arr[k]
    field["mlp"] = {k[4:]: arr[k] for k in arr if k.startswith("mlp_")}
    return field

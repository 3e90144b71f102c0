"""Reader for the small text fixtures in this folder (values printed in the paper)."""

import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _num(tok):
    neg = tok.startswith("-")
    body = tok[1:] if neg else tok
    v = math.sqrt(2.0) if body == "r2" else float(body)
    return -v if neg else v


def load(name):
    out = {}
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(":")
            out[key.strip()] = [_num(t) for t in rest.split()]
    return out

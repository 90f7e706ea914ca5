"""Result lines and arrays of the GPU tests: always printed; also appended to
$FW25_REPORT_DIR/parity.txt (arrays saved there) when that variable names a
directory to collect them in."""
import os

import numpy as np


def _dir():
    d = os.environ.get("FW25_REPORT_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
    return d


def report(line):
    d = _dir()
    if d:
        with open(os.path.join(d, "parity.txt"), "a") as fh:
            fh.write(line + "\n")
    print(line, flush=True)


def save(name, array):
    d = _dir()
    if d:
        np.save(os.path.join(d, name), array)

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle test that takes tens of seconds on the CPU")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(v):
    try:
        return float(v)
    except ValueError:
        return v


def load_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([_num(v) for v in line.split()])
    return rows


def load_table_raw(name):
    """Rows of the golden file as the printed strings (to recover the printed precision)."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def printed_half_unit(s):
    """Half a unit in the last printed digit of a decimal string such as '0.1367' or '4.6592E-01'."""
    mant, _, exp = s.upper().partition("E")
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (-decimals + (int(exp) if exp else 0))

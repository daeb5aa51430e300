"""Helpers shared by the tests (no method arithmetic)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_09543_amd", "libntbc.so")


def ensure_built():
    """Builds libntbc.so if it is missing (tests load what is built)."""
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, "-m", "paper_2407_09543_amd.build"], cwd=ROOT, check=True)
    return LIB


def u64(t):
    """int64 torch tensor (BC words) -> numpy uint64 on the host."""
    return t.detach().cpu().numpy().view(np.uint64)


def log(msg):
    print(msg, flush=True)

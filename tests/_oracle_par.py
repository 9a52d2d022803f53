"""The CPU oracle over a large lane range, split into chunks on host threads
(the oracle's ctypes calls release the GIL, so the chunks run in parallel).
Each chunk is the oracle's own function on lanes [s0, s1) with i0 = s0, so
the result is exactly the oracle's for the whole range."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def threads():
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def by_chunks(fn, n, chunk=1 << 18):
    """fn(s0, s1) -> float32[s1 - s0] for every chunk of [0, n), concatenated."""
    bounds = [(s, min(n, s + chunk)) for s in range(0, n, chunk)]
    out = np.empty(n, np.float32)
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        for (s0, s1), part in zip(bounds, ex.map(lambda b: fn(*b), bounds)):
            out[s0:s1] = part
    return out

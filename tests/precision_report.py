"""Per-output error table against the FP64 oracle.

When the environment variable GM_PRECISION_REPORT names a file, the GPU parity tests that call
row() append one markdown table row per output to it (the header is written first if the file
is new); otherwise row() does nothing.  Each row gives, for the GPU output against the oracle's:
  normwise    max |gpu - ref| / max |ref|   (the bar the tests hold: 1e-5 FP32, 2e-2 BF16)
  p50, p99    quantiles of |gpu - ref| / max |ref| over the elements
  rel         max |gpu - ref| / |ref| over the elements with |ref| >= 1e-3 max |ref|; it
              grows without bound where an output passes through zero (an absolute error of
              the output's own scale divided by a small value), so it is reported, not held
"""
import os

import numpy as np

HEADER = ("| workload | output | arithmetic | elements | normwise | p50 | p99 | rel (|ref| >= 1e-3 max) |\n"
          "|---|---|---|---|---|---|---|---|\n")


def row(workload, output, arithmetic, got, ref):
    path = os.environ.get("GM_PRECISION_REPORT")
    if not path:
        return
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    s = float(np.max(np.abs(ref))) if ref.size else 0.0
    d = np.abs(got - ref)
    if s > 0:
        q = d / s
        big = np.abs(ref) >= 1e-3 * s
        rel = float(np.max(d[big] / np.abs(ref[big])))
        cells = [f"{float(np.max(q)):.2e}", f"{float(np.percentile(q, 50)):.2e}",
                 f"{float(np.percentile(q, 99)):.2e}", f"{rel:.2e}"]
    else:
        cells = [f"{float(np.max(d)) if d.size else 0.0:.2e} (abs)", "-", "-", "-"]
    new = not os.path.exists(path)
    with open(path, "a") as f:
        if new:
            f.write(HEADER)
        f.write(f"| {workload} | {output} | {arithmetic} | {ref.size} | " + " | ".join(cells) + " |\n")

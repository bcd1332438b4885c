"""Run the oracle's compensated sums (Sec. 4: the 6-operation and the
3-operation form) over every pair of finite fp16 values and every pair of
finite bf16 values, and store the counts of pairs that are not error free.

    python tests/golden/make_eft_exhaustive.py

Output: eft_exhaustive.json next to this file (counts as named by
oracle.EFT_COUNTS, per format, and the seconds taken).  Calls only the
oracle.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402


def main():
    out = {"what": "every pair (a, b) of finite values of the format; a + b = s + t "
                   "checked exactly for the 6-operation sum (all pairs) and the "
                   "3-operation sum (pairs with |a| >= |b|); pairs where an "
                   "operation overflows are counted apart",
           "threads": oracle.max_threads()}
    for fmt in ("f16", "bf16"):
        t = time.time()
        c = oracle.eft_exhaustive(fmt)
        c["seconds"] = round(time.time() - t, 1)
        out[fmt] = c
        print(fmt, c, flush=True)
    with open(os.path.join(HERE, "eft_exhaustive.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()

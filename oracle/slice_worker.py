"""One single-threaded oracle process scoring a slice of the rung-3 workload
(test and benchmark infrastructure only; imports no GPU library).

    python -m oracle.slice_worker SEED BEGIN END

builds the seeded rung-3 problem (n = 2000, d = 20) and scores ids
[BEGIN, END) of its space against y with the FP64 oracle, then prints the
number of ids and the elapsed seconds of the scoring alone.
"""
import sys
import time

from oracle import oracle as O
from paper_2410_01752_amd import inputs as I


def main():
    seed, begin, end = int(sys.argv[1]), int(sys.argv[2]), int(sys.argv[3])
    p = I.config3(seed=seed)
    sp = O.Space(p.X.shape[1], p.unary, p.binary, p.rung, p.rect)
    t0 = time.perf_counter()
    sp.score_range(p.X, p.y, begin, end)
    print(end - begin, time.perf_counter() - t0, flush=True)


if __name__ == "__main__":
    main()

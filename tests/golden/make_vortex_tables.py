"""Write tests/golden/vortex_oracle_tables.txt: the oracle's moving-vortex
errors at T = 2 on every mesh and degree of Tables 1 and 2 (Sec. 6.1).

Calls only the oracle (oracle/box.py) and the input generator.  The
eta_Linf column is the largest nodal error, which is not the paper's L_inf
(see tests/test_oracle_box.py).  Runs the 16 cases in worker processes;
the 32x32, p = 5 case (3200 steps) takes the longest.

    python tests/golden/make_vortex_tables.py [workers]
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

CASES = [(p, n) for p in (2, 3, 4, 5) for n in (4, 8, 16, 32)]


def one(case):
    from test_oracle_box import run_vortex
    p, n = case
    t0 = time.time()
    e = run_vortex(p, n)
    return case, e, time.time() - t0


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    out = {}
    # longest first
    order = sorted(CASES, key=lambda c: -(c[1] ** 2) * (c[0] + 1) ** 2 * 2 ** c[0])
    with ProcessPoolExecutor(workers) as ex:
        for (p, n), e, dt in ex.map(one, order):
            out[(p, n)] = e
            print(f"p={p} n={n}: {dt:.0f} s", flush=True)
    with open(os.path.join(HERE, "vortex_oracle_tables.txt"), "w") as f:
        f.write("# Oracle (oracle/box.py) errors of the moving vortex at T = 2, written by\n"
                "# tests/golden/make_vortex_tables.py; columns as in vortex_tables.txt,\n"
                "# except eta_Linf: the largest nodal error.\n"
                "# p  n   eta_L1     eta_L2     eta_Linf   u_L2       v_L2       sqrtE\n")
        for p, n in CASES:
            e = out[(p, n)]
            f.write(f"{p}  {n:2d}   " + "  ".join(f"{e[c]:.6e}" for c in
                    ("eta_L1", "eta_L2", "eta_Linf_nodes", "u_L2", "v_L2", "sqrtE")) + "\n")


if __name__ == "__main__":
    main()

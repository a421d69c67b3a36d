"""Write channel_study_nx64.txt: the FP64 oracle's flux of eq. (11) in rough
channels of the paper's two widths (steps a = 8, b = 4, p = 32 on both walls,
64 columns: two whole periods), after a fixed 300 000 steps from the seeded
cold start, for
  - the configs' normalisation (reading R1, G = -5, tau = 1, two-node layer),
    widths 80 and 160, fields 0, 1.5e-3, 3e-3;
  - the paper's own parameters (reading R29, calG = -0.52, w = -0.14,
    tau = 0.9, f_b = 8e-6, single-node layer), width 80, fields 0, 0.05, 0.1.

Only the oracle and the seeded input generators are used.  One single-thread
process per channel; about 6 minutes on 8 cores.  Run from the repository root:
    python tests/golden/make_channel_study.py
"""
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

NX = 64
STEPS = 300_000
CHUNK = 2000
CASES = [("configs", w, f) for w in (80, 160) for f in (0.0, 1.5e-3, 3e-3)] + \
        [("paper", 80, f) for f in (0.0, 0.05, 0.1)]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "channel_study_nx64.txt")


def case(reading, w, f):
    from paper_0708_4182_amd import inputs as I
    if reading == "paper":
        return I.paper_channel_case(nx=NX, ny=w, f_elec=f, seed=0)
    return I.rough_channel_case(nx=NX, ny=w, f_elec=f, seed=0, layers=2)


def run(key):
    import oracle as O
    O.threads(1)
    c = case(*key)
    f = O.init(c.params, c.solid, c.rho)
    last = []
    for k in range(STEPS // CHUNK):
        O.step(c.params, c.solid, f, CHUNK)
        if k >= STEPS // CHUNK - 3:
            last.append(O.flux(c.params, c.solid, f)[0])
    Q, M = O.flux(c.params, c.solid, f)
    return key, Q, M, abs(last[-1] - last[0]) / abs(last[-1])


def main():
    with Pool(min(8, len(CASES))) as pool:
        rows = pool.map(run, CASES)
    with open(OUT, "w") as fh:
        fh.write(f"# FP64 oracle, rough-wall channels {NX} x width (a=8, b=4, p=32, seed 0), cold start,\n")
        fh.write(f"# {STEPS} steps; flux Q and mass M of eq. (11) over fluid nodes.\n")
        fh.write("# Written by tests/golden/make_channel_study.py.  drift = |dQ| / Q over the last 4000 steps.\n")
        fh.write("# columns: reading  width  f_elec  Q  M  drift\n")
        for (reading, w, f), Q, M, d in rows:
            fh.write(f"{reading} {w} {f:g} {Q!r} {M!r} {d:.3e}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()

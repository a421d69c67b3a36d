"""Write the input file of the standalone profiling driver (csrc/step_driver.cpp):
    python -m paper_0708_4182_amd.profile_case OUT [nx ny]
the benchmark's random-step rough channel (default 8192 x 2048, seed 0,
f = 1e-3): int32 nx, ny; the lbm_params struct; uint8 solid [ny][nx];
float64 initial density [ny][nx]."""
from __future__ import annotations

import sys

import numpy as np

from . import inputs as I
from . import lbm


def main(argv):
    out = argv[1]
    nx, ny = (int(argv[2]), int(argv[3])) if len(argv) > 3 else (8192, 2048)
    c = I.random_channel_case(nx=nx, ny=ny, f_elec=1e-3, seed=0)
    p = lbm.to_c_params(c.params)
    with open(out, "wb") as fh:
        fh.write(np.array([nx, ny], np.int32).tobytes())
        fh.write(bytes(p))
        fh.write(np.ascontiguousarray(c.solid, np.uint8).tobytes())
        fh.write(np.ascontiguousarray(c.rho, np.float64).tobytes())
    print(f"wrote {out}: {nx} x {ny}, {int((c.solid == 0).sum())} fluid nodes")


if __name__ == "__main__":
    main(sys.argv)

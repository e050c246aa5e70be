"""Write the synthetic observed spectra synth/data/obs_c{N}.txt from the FP64 oracle.

y_k = (binned oracle model at the seeded truth parameters)_k + N(0, 50 ppm)_k.
Only the oracle computes the model here; the files are inputs shared by the
oracle and the HIP library.  Run: python tests/golden/make_obs.py [cid ...]
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import synth  # noqa: E402
import oracle  # noqa: E402


def main(cids):
    for cid in cids:
        wl = synth.workload(cid, batch=1, require_obs=False)
        theta = synth.truth_params(cid)
        n_lay = wl["n_layers"] if wl["n_layers_per_sample"] is None else 100
        out = oracle.forward(wl, theta, n_layers=n_lay)
        if out["status"]:
            raise RuntimeError(f"truth sample of config {cid} is invalid: status {out['status']}")
        y = out["binned"] + synth.noise(cid, len(wl["bin_lo"]), wl["sigma_ppm"])
        path = synth.obs_path(cid)
        np.savetxt(path, y, fmt="%.17e",
                   header=f"config {cid}: binned FP64 oracle model at the seeded truth parameters "
                          f"{np.array2string(theta, precision=6)} plus N(0, {wl['sigma_ppm']} ppm) noise")
        print(cid, path, y[:3])


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [0, 1, 2, 3, 4, 5, 6])

"""Write the stored reference answers used by the benchmark and the
full-size GPU tests. Calls only the oracle and the seeded generators.

    python tests/golden/make_golden.py            # the workloads
    python tests/golden/make_golden.py examples   # the paper's five problems

For each workload: the plain float64 RQI-PCGTLS of the oracle (Algorithms
2 and 3), its Rayleigh quotient re-evaluated in long double, Newton
polishing with long-double residuals, and the certificates of
oracle.certify (normal-equation residual, smallest root). The file records
the certificate values next to the answer.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tlsgen  # noqa: E402
from oracle import certify, polish, rqi  # noqa: E402

WORKLOADS = {
    # name: (generator call, description)
    "sparse_c2": (lambda: tlsgen.sparse_scaled(20000, 2000, 0.005, 4.0, 1e-4, seed=2000)[:2],
                  "CSR 20000x2000, 0.5% nnz, column scales logU[1,1e4], b noise 1e-4, seed 2000"),
    "dense_c1": (lambda: tlsgen.dense_gaussian(200, 20, seed=1000)[:2],
                 "dense 200x20 N(0,1) + 1e-3 perturbation, b noise 1e-3, seed 1000"),
    "dense_c3": (lambda: tlsgen.reflector_dense(65536, 4096, seed=3000)[:2],
                 "dense 65536x4096 = Y diag(s) Z^T + E, single reflectors Y, Z, s geometric "
                 "1..1e-3, E spectral size 1e-5, b noise 1e-5, seed 3000"),
}
# written only when named on the command line (minutes of CPU time)
ON_REQUEST = {"dense_c3"}


def reference(name, bounds=False):
    A, b = WORKLOADS[name][0]()
    t0 = time.time()
    res = rqi.rqi_pcgtls(A, b, patience=2)
    x, sig = polish.polish(A, b, res.x, steps=2)
    c = certify.certify(A, b, x, sig)
    out = {
        "workload": name,
        "description": WORKLOADS[name][1],
        "sigma": sig,
        "x": [float(v) for v in x],
        "certificate": {"normal_eq": c.normal_eq, "g_rel": c.g_rel, "rq_rel": c.rq_rel,
                        "smallest_root": bool(c.smallest_root)},
        "oracle_iters": res.iters,
        "oracle_seconds": time.time() - t0,
    }
    if bounds:
        # attainable float64 accuracy (Section 1): sigma'_1, sigma'_n from the
        # eigenvalues of A^T A, sigma_1([A, b]) from those of [A, b]^T [A, b]
        G = rqi.gram(A)
        ev = np.linalg.eigvalsh(G)
        s1, sn = float(np.sqrt(ev[-1])), float(np.sqrt(ev[0]))
        Atb = np.asarray(A).T @ b
        Gb = np.block([[G, Atb[:, None]], [Atb[None, :], np.array([[b @ b]])]])
        s1ab = float(np.sqrt(np.linalg.eigvalsh(Gb)[-1]))
        ktls = certify.kappa_tls(s1, sn, sig)
        bs, bx = certify.attainable(s1ab, sig, ktls)
        out["bounds"] = {"sigma_1_A": s1, "sigma_n_A": sn, "sigma_1_Ab": s1ab, "kappa_tls": ktls,
                         "existence_margin": certify.existence_margin(sn, sig),
                         "attainable_sigma": bs, "attainable_x": bx}
    return out


# the five problems of Section 4, answered in extended precision (50-digit
# mpmath eigen-decomposition of [A, b]^T [A, b]) for the error curves
EXAMPLES = ["paper_random", "paper_delta", "paper_toeplitz", "paper_vanhuffel", "paper_bjorck"]


def examples():
    from oracle import exact
    out = {}
    for gen in EXAMPLES:
        A, b = getattr(tlsgen, gen)()[:2]
        t0 = time.time()
        r = exact.mp_svd_tls(A, b)
        out[gen] = {"sigma": float(r.sigma), "x": [float(v) for v in r.x],
                    "sigma_1_Ab": float(r.sigma_1_Ab), "kappa_tls": float(r.kappa_tls),
                    "seconds": time.time() - t0}
        print(gen, "sigma", out[gen]["sigma"], f"{out[gen]['seconds']:.1f}s", flush=True)
    with open(os.path.join(HERE, "paper_examples_mp.json"), "w") as f:
        json.dump(out, f, indent=0)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "examples":
        examples()
        return
    names = sys.argv[1:] or [w for w in WORKLOADS if w not in ON_REQUEST]
    for name in names:
        ref = reference(name, bounds=name in ON_REQUEST)
        path = os.path.join(HERE, f"{name}_ref.json")
        with open(path, "w") as f:
            json.dump(ref, f, indent=0)
        print(name, "sigma", ref["sigma"], ref["certificate"], f"{ref['oracle_seconds']:.2f}s")


if __name__ == "__main__":
    main()

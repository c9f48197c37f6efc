"""Writes tests/golden/oracle_<workload>.json: the FP64 oracle's PBM result on
a benchmark workload (compliance 1/2 f^T u, exact compliance of the final
density by a sparse direct solve, KKT terms, duality certificate, iteration
counts and the per-step logs of Algorithms 1 and 2).  Calls only oracle/ and
workloads/; the GPU path is not involved.

    python tests/golden/make_oracle_results.py 1        # the 64x32x32 cantilever

Takes about half an hour on one core for the 64x32x32 cantilever.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


import workloads as W  # noqa: E402
from oracle import kkt, pbm  # noqa: E402


def main(idx: int):
    pr = W.config(idx)
    opts = pbm.Options()
    if pr.extra.get("eps_mr0"):
        opts.eps_mr0 = pr.extra["eps_mr0"]
    t0 = time.time()
    s = pbm.Solver(pr, opts)
    s.progress = lambda k, d: print(f"outer {k}: ratio {d['ratio']:.3e} stat {d['stat']:.3e} "
                                    f"newton so far {len(s.log.newton)} "
                                    f"({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    st = s.solve()
    t1 = time.time()
    P = s.P
    r = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho, st.u, st.alpha)
    c_exact = kkt.compliance(P.grid, P.Ke, st.rho, P.f)
    lb, ub, cert = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho, st.u)
    out = dict(workload=pr.name, status=s.status, seconds=t1 - t0,
               compliance_half_fu=float(0.5 * P.f @ st.u), compliance_exact=float(c_exact),
               certificate_lower=float(lb), certificate_upper=float(ub), certificate_rel=float(cert),
               alpha=float(st.alpha), sum_rho=float(st.rho.sum()), V=P.V,
               outer=len(s.log.outer), newton=len(s.log.newton),
               minres=int(sum(d["minres"] for d in s.log.newton)),
               options={k: getattr(opts, k) for k in vars(opts)},
               newton_log=s.log.newton, outer_log=s.log.outer, **r)
    path = os.path.join(HERE, f"oracle_{pr.name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1)

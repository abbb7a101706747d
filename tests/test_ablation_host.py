"""The paper's conditioning-schedule example (Sec. IV, Fig. 2) with the oracle:
10 random LPs (80 x 100), t = 9.2, and the three schedules L = {} (no
conditioning), L = {300} and L = {1, ..., 50}.  The paper's qualitative
finding: a single conditioning already speeds convergence up substantially.
This pins the conditioning steps (5-14) against the paper's own claim: a
wrong ratio, exponent or re-cast of s would not give the ordering."""
import numpy as np

from oracle.alg2 import Algorithm2, Schedule
from paper_2103_00736_amd import synth

SCHEDULES = {"none": Schedule(0, 0, -1), "once_300": Schedule(300, 0, -1), "first_50": Schedule(1, 1, 50)}


def iterations_to(eps, sched, index, cap=20000):
    p = synth.e2_lp(index)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=9.2, schedule=sched)
    alg.run(cap, eps=eps, check_every=10)
    return alg.l


def test_conditioning_schedules_order_as_in_the_paper():
    its = {k: [iterations_to(1e-6, s, i) for i in range(10)] for k, s in SCHEDULES.items()}
    med = {k: float(np.median(v)) for k, v in its.items()}
    print(its, med)
    assert med["once_300"] < 0.25 * med["none"]
    assert med["first_50"] < med["once_300"]
    # conditioning at l = 300 cannot help before 300 iterations: no run stops earlier
    assert min(its["once_300"]) >= 300 or min(its["once_300"]) == min(its["none"])

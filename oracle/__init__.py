"""FP64 CPU oracle of the penalised market-surplus objective, its gradient and
the modified Adam step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the HIP library; the two meet only in the seeded input
generator, which draws numbers and computes none of the method.

Modules
-------
network    DC network algebra: incidence, bridges by brute force, the
           reduced-susceptance solve (eqs. (Yb_solve), (p_flow)), injection
           shift factors and line outage distribution factors, and the
           per-outage re-solve that defines a contingency flow.
objective  the objective terms and their manual reverse pass (Section II,
           eqs. (nlp_updated), (grads)), in a fast LODF form and a
           brute-force contingency form.
adam       the step-size schedule (eqs. (norm_t)-(step_size)) and the
           modified Adam update with clipping (Alg. 3).
solve      a plain Adam loop over the two above (the Adam window of Alg. 4).

Readings of the paper that this oracle fixes where the text is silent are
listed in each module's header.
"""

"""FP64 CPU oracle for Monte Carlo valuation of compiled payoff expressions.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the GPU library is checked against.  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product library never does, and this package
imports nothing from the product library.  The two share no code: the only
common module is ``workloads`` (seeded input generators, which hold none of
the method's arithmetic).

What it computes (Annenkov & Elsman, "Certified Compilation of Financial
Contracts", PPDP'18):

* ``il``      -- the payoff intermediate language: syntax (Sec. 3 grammar and
                 the Coq ``ILExpr``/``ILTExpr``/``ILTExprZ`` types of Sec. 5),
                 a type check (the value domain N + R + B of Fig. 3; Thm. 2 is
                 the guarantee that well-typed compiled IL evaluates), and the
                 denotational semantics of Fig. 3.
* ``grid``    -- the days an expression can read (the horizon bound HOR of
                 Sec. 4 and the time re-indexing of the Futhark backend,
                 Sec. 6.2).
* ``rng``     -- Philox4x32-10 (Salmon et al., SC'11) and unscrambled Sobol
                 points (scipy), with the exact dyadic uniform maps.
* ``model``   -- risk-neutral correlated GBM paths (textbook Cholesky,
                 log-Euler steps).
* ``mc``      -- the Monte Carlo estimator: paths, per-path payoff values,
                 mean and standard error.
* ``closed_form`` -- Black-Scholes and barrier closed forms used as pins.
* ``mlp``     -- FP64 numpy MLP (forward, backward, Adam) for the surrogate.

Every floating-point step is IEEE double.  Functions cite the passage of the
paper they follow; where the paper is silent the docstring names the reading
taken.
"""

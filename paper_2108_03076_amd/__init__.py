"""MI355X-native Monte Carlo valuation of compiled payoff expressions.

The library (libpmc.so, C ABI in include/pmc.h) loads a payoff expression of
the payoff intermediate language of Annenkov & Elsman, "Certified
Compilation of Financial Contracts" (Sec. 3, Fig. 3), and prices it by Monte
Carlo on one gfx950 GPU: counter-based or quasi-random numbers, inverse-CDF
normals, correlated GBM steps over the expression's dates, the payoff
interpreted per path, and one FP64 sum over paths.  This package is the
Python binding (argument marshalling only); torch supplies device memory
and streams.
"""
from ._lib import (EXPORTED, LIB_PATH, Context, PmcError, Payoff, autotune_batch, compile_contract, eval_paths,
                   gen_paths, load_contract,
                   lib, load_payoff, price, price_batch, price_noalloc, risk_batch, Pricer, BatchPricer, Surrogate)

__all__ = ["Context", "Payoff", "PmcError", "price", "price_batch", "price_noalloc", "risk_batch", "autotune_batch", "gen_paths",
           "eval_paths", "load_payoff", "compile_contract", "load_contract", "Pricer", "BatchPricer", "Surrogate", "lib", "LIB_PATH", "EXPORTED"]

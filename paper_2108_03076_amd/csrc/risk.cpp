// Bump-and-revalue risk on common random numbers: expands every instance of
// a batch into its 1 + 4A scenarios (base; S_a +- h_a; sigma_a +- k), prices
// them all in one persistent batch launch with the instance's own stream id,
// and forms central differences.
#include <cmath>
#include <string>
#include <vector>

#include "../../include/pmc.h"
#include "ctx.h"

using namespace pmc;

extern "C" int pmc_risk_batch(pmc_ctx* c, const pmc_payoff* p, const pmc_batch* b, const pmc_gbm* m,
                              const pmc_opts* o, const pmc_risk_opts* r, pmc_greeks* out) {
  if (!c || !p || !b || !m || !o || !r || !out) return ctx_fail(c, PMC_E_ARG, "null argument");
  pmc_payoff_info info{};
  int st = pmc_payoff_get_info(p, &info);
  if (st != PMC_OK) return ctx_fail(c, st, "payoff info");
  const int A = info.n_assets, V = info.n_tvars, Q = info.n_params;
  const int I = b->n_inst;
  if (I < 1) return ctx_fail(c, PMC_E_ARG, "n_inst must be >= 1");
  if (b->per_instance_model ? (!b->spot || !b->vol) : (!m->spot || !m->vol))
    return ctx_fail(c, PMC_E_ARG, "model spot and vol are required");
  if (o->history)   // the simulation would start from the history, not the bumped spots
    return ctx_fail(c, PMC_E_UNSUPPORTED, "risk runs do not take a price history");
  const double rel = r->rel_spot_bump, k = r->abs_vol_bump;
  if (!(rel > 0.0 && rel < 1.0) || !(k > 0.0) || !std::isfinite(k))
    return ctx_fail(c, PMC_E_ARG, "bumps must satisfy 0 < rel_spot_bump < 1 and abs_vol_bump > 0");
  const int S = 1 + 4 * A;
  const size_t n = (size_t)I * S;
  if (n > 0x7fffffffu) return ctx_fail(c, PMC_E_UNSUPPORTED, "too many scenarios");
  std::vector<int32_t> tenv(n * V);
  std::vector<double> params(n * Q), spot(n * A), vol(n * A), corr(n * A * A);
  std::vector<uint32_t> ids(n);
  for (int i = 0; i < I; ++i) {
    const double* s0 = b->per_instance_model ? b->spot + (size_t)i * A : m->spot;
    const double* v0 = b->per_instance_model ? b->vol + (size_t)i * A : m->vol;
    const double* c0 = b->per_instance_model ? (b->corr ? b->corr + (size_t)i * A * A : nullptr) : m->corr;
    for (int a = 0; a < A; ++a)
      if (!(v0[a] > k)) return ctx_fail(c, PMC_E_ARG, "abs_vol_bump must be below every volatility");
    for (int j = 0; j < S; ++j) {
      const size_t e = (size_t)i * S + j;
      for (int t = 0; t < V; ++t) tenv[e * V + t] = b->tenv ? b->tenv[(size_t)i * V + t] : 0;
      for (int q = 0; q < Q; ++q) params[e * Q + q] = b->params ? b->params[(size_t)i * Q + q] : 0.0;
      for (int a = 0; a < A; ++a) { spot[e * A + a] = s0[a]; vol[e * A + a] = v0[a]; }
      for (int x = 0; x < A * A; ++x) corr[e * A * A + x] = c0 ? c0[x] : (x % (A + 1) == 0 ? 1.0 : 0.0);
      ids[e] = b->instance_ids ? b->instance_ids[i] : (uint32_t)i;
      if (j >= 1 && j <= 2 * A) {            // spot pair of asset (j-1)/2
        const int a = (j - 1) / 2;
        spot[e * A + a] = s0[a] + ((j - 1) % 2 == 0 ? 1.0 : -1.0) * rel * s0[a];
      } else if (j > 2 * A) {                // volatility pair of asset (j-1-2A)/2
        const int a = (j - 1 - 2 * A) / 2;
        vol[e * A + a] = v0[a] + ((j - 1 - 2 * A) % 2 == 0 ? 1.0 : -1.0) * k;
      }
    }
  }
  pmc_batch eb{};
  eb.n_inst = (int)n;
  eb.tenv = V ? tenv.data() : nullptr;
  eb.params = Q ? params.data() : nullptr;
  eb.per_instance_model = 1;
  eb.spot = spot.data();
  eb.vol = vol.data();
  eb.corr = corr.data();
  eb.instance_ids = ids.data();
  std::vector<pmc_result> res(n);
  st = pmc_price_batch(c, p, &eb, m, o, res.data());
  if (st != PMC_OK) return st;
  for (int i = 0; i < I; ++i) {
    const pmc_result* R = res.data() + (size_t)i * S;
    pmc_greeks g{};
    g.price = R[0].price;
    g.std_err = R[0].std_err;
    const double* s0 = b->per_instance_model ? b->spot + (size_t)i * A : m->spot;
    for (int a = 0; a < A; ++a) {
      const double h = rel * s0[a];
      const double up = R[1 + 2 * a].price, dn = R[2 + 2 * a].price;
      g.delta[a] = (up - dn) / (2.0 * h);
      g.gamma[a] = (up - 2.0 * g.price + dn) / (h * h);
      const double vu = R[1 + 2 * A + 2 * a].price, vd = R[2 + 2 * A + 2 * a].price;
      g.vega[a] = (vu - vd) / (2.0 * k);
    }
    g.ms = R[0].ms;
    out[i] = g;
  }
  return PMC_OK;
}

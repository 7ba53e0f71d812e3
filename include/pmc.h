/*
 * pmc.h -- C ABI of libpmc: Monte Carlo valuation of compiled payoff
 * expressions on one MI355X (gfx950) GPU.
 *
 * The method is that of Annenkov & Elsman, "Certified Compilation of
 * Financial Contracts" (PPDP'18): contracts are compiled to a payoff
 * intermediate language (IL, Sec. 3, Fig. 3), and a pricing engine
 * evaluates the payoff expression on simulated scenarios of the external
 * environment and aggregates the discounted value (Sec. 3, Sec. 6.2).  The
 * engine is parameterised by the compiled payoff, so one expression is
 * loaded once and priced for many template environments, parameters and
 * models (Sec. 6.2; templates and instruments, Sec. 2).
 *
 * Conventions for every entry point:
 *   - Return value: PMC_OK (0) or a negative pmc_status.  On error nothing
 *     is written to output arguments and pmc_last_error() describes it.
 *     No entry point aborts the process.
 *   - Host pointers are read during the call only (copied); the caller
 *     keeps ownership.  Device pointers (suffix _dev) are caller-owned
 *     device memory on the context's device; they must stay valid until
 *     the call returns (every call synchronises the context's stream before
 *     it returns).
 *   - A pmc_ctx is bound to one device and one HIP stream and must not be
 *     used from two threads at once.  A pmc_payoff is immutable after load
 *     and may be used with any context on the same device.
 *
 * IL text syntax (S-expressions; one form per IL constructor of Fig. 3 and
 * the Coq ILExpr type of Sec. 5):
 *   e  ::= (now) | (real F) | (nat N) | (bool true|false) | (t T)
 *        | (model LABEL Z) | (payoff T P1 P2)
 *        | (if e e e) | (loopif e e e T)
 *        | (neg e) | (not e) | (OP e e)
 *   OP ::= add | sub | mult | div | min | max | lt | leq | eq | and | or
 *   T  ::= N | (tvar NAME) | (tplus T T)          -- ILTExpr
 *   Z  ::= T | (int I) | (tplusz Z Z)             -- ILTExprZ
 * Value types: N (naturals: now, nat, t), R (reals: real, model, payoff and
 * arithmetic), B (booleans).  add/min/max work on N or R; sub/mult/div on R;
 * lt/leq on N or R; eq on equal types; and/or/not on B; neg on R.
 * Semantics (Fig. 3): (t T) is T + t0; (model l Z) is the observable l on
 * day Z + t0; (payoff T p q) is +d(T + t0) if (p,q) = (from,to), -d(T + t0)
 * if (p,q) = (to,from), else 0; (loopif c a b n) checks c on days
 * t0 .. t0+n and gives a on the first day it holds, else b on day t0+n.
 * Observables: asset labels are simulated prices (day <= 0 is the spot);
 * parameter labels are constants (e.g. strike, barrier).
 */
#ifndef PMC_H_
#define PMC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmc_ctx pmc_ctx;
typedef struct pmc_payoff pmc_payoff;

typedef enum pmc_status {
  PMC_OK = 0,
  PMC_E_ARG = -1,          /* bad argument (NULL, out of range, NaN/Inf) */
  PMC_E_PARSE = -2,        /* IL text does not follow the grammar above */
  PMC_E_TYPE = -3,         /* ill-typed IL (Thm. 2 needs well-typed IL) */
  PMC_E_TENV = -4,         /* template variable unbound or negative */
  PMC_E_HORIZON = -5,      /* a read day beyond PMC_MAX_HORIZON */
  PMC_E_NOT_PD = -6,       /* correlation matrix not positive definite */
  PMC_E_UNSUPPORTED = -7,  /* beyond a documented limit below */
  PMC_E_HIP = -8,          /* HIP runtime error */
  PMC_E_OOM = -9           /* device or host allocation failed */
} pmc_status;

#define PMC_MAX_ASSETS 4
#define PMC_MAX_HORIZON 65536
#define PMC_MAX_LOOP_DEPTH 8
#define PMC_MAX_REGS 31

enum { PMC_RNG_PHILOX = 0, PMC_RNG_SOBOL = 1 };
enum { PMC_FP32 = 0, PMC_FP64 = 1 };
enum { PMC_MODE_AUTO = 0, PMC_MODE_TWO_PHASE = 1, PMC_MODE_FUSED = 2 };
/* Payoff engines: the bytecode interpreter (wavefront-uniform program
 * counter) or the payoff compiled to a device function at run time (hipRTC;
 * the first price call of a payoff/precision/rng variant compiles it, which
 * takes seconds; later calls reuse it).  AUTO selects COMPILED. */
enum { PMC_ENGINE_AUTO = 0, PMC_ENGINE_INTERPRETER = 1, PMC_ENGINE_COMPILED = 2 };

/* Library version string (static storage). */
const char* pmc_version(void);

/* Create a context on HIP device `device` using HIP stream `hip_stream`
 * (a hipStream_t; NULL means the null stream).  *out receives the handle. */
int pmc_ctx_create(int device, void* hip_stream, pmc_ctx** out);
void pmc_ctx_destroy(pmc_ctx* ctx);
/* Text of the last error on this context (owned by ctx; valid until the
 * next call on it); with ctx == NULL, the last error of a context-free call
 * on this thread.  Never NULL. */
const char* pmc_last_error(const pmc_ctx* ctx);

/* Load a compiled payoff expression (Sec. 3 IL; the engine "compiles once
 * per instrument", Sec. 6.2).  ctx may be NULL (loading needs no device).
 * il_text need not be NUL-terminated (len
 * bytes).  asset_labels[n_assets] name the simulated observables in model
 * order (1 <= n_assets <= PMC_MAX_ASSETS); param_labels[n_params] name the
 * constant parameter observables (strike etc.; the paper keeps non-temporal
 * parameters as constant observables, Sec. 2 footnote); tvar_names[n_tvars]
 * fix the order of template variables in every tenv array (Sec. 2,
 * TEnv : Var -> N).  The text is parsed, type-checked and encoded to
 * bytecode.  Errors: PMC_E_PARSE, PMC_E_TYPE (also for a model label that is
 * neither an asset nor a parameter), PMC_E_UNSUPPORTED (expression needs
 * more than PMC_MAX_REGS registers or PMC_MAX_LOOP_DEPTH nested loopifs). */
int pmc_payoff_load(pmc_ctx* ctx, const char* il_text, size_t len,
                    const char* const* asset_labels, int n_assets,
                    const char* const* param_labels, int n_params,
                    const char* const* tvar_names, int n_tvars, pmc_payoff** out);
void pmc_payoff_free(pmc_payoff* p);

/* Contract language (CL) front end (Sec. 2, Fig. 1, with template
 * expressions; Sec. 4, the compilation tau_c / tau_e).  Contract text:
 *   c ::= zero | transfer(P1, P2 [, ASSET]) | scale(e, c) | translate(t, c)
 *       | ifWithin(e, t, c, c) | if(e, c, c) | both(c, c) | all[c, ..., c]
 *   t ::= N | NAME                      (a numeral or a template variable)
 *   e ::= obs(LABEL, I) | F | true | false | (e) | -e | !e
 *       | e OP e   with OP, loosest first: || ; && ; < <= > >= == ; + - ; * /
 *       | add|sub|mult|div|min|max|lt|leq|eq|and|or(e, e) | neg|not(e)
 *       | cond(e, e, e)
 * if(e, c1, c2) is ifWithin(e, 0, c1, c2) (checked at the current time
 * only); all[c1, ..., cn] abbreviates both(c1, both(..., cn)); ';' starts a
 * comment to the end of the line.  The asset of a transfer is dropped
 * (one currency, two-party view).  Compilation accumulates translate's
 * shifts into the start time t0 with the smart addition of Sec. 4
 * (numerals are added; the numeral 0 is the identity): obs(l, i) becomes
 * (model l t0+i), transfer (payoff t0 P1 P2), scale mult, both add, zero
 * (real 0.0), cond and if (if ...), ifWithin (loopif e c1 c2 t), and the
 * comparisons > and >= become lt and leq with their operands swapped.
 * pmc_contract_compile writes the payoff-language text (at most cap bytes,
 * NUL-terminated; *il_len gets the full length; il_out may be NULL to
 * query).  pmc_contract_load compiles and loads it as pmc_payoff_load
 * does, with the same label arguments (observables in obs(l, i) are asset
 * or parameter labels; template variables in t are tvar_names).
 * Times and observation offsets are numerals below 2^31 (days); contracts
 * and expressions nest at most 1000 deep.
 * Errors: PMC_E_PARSE (contract syntax, a numeral out of range, nesting
 * beyond the limit; with the offset in pmc_last_error), and those of
 * pmc_payoff_load. */
int pmc_contract_compile(const char* cl_text, size_t len, char* il_out, size_t cap, size_t* il_len);
int pmc_contract_load(pmc_ctx* ctx, const char* cl_text, size_t len,
                      const char* const* asset_labels, int n_assets,
                      const char* const* param_labels, int n_params,
                      const char* const* tvar_names, int n_tvars, pmc_payoff** out);

/* Time-parameterised payoff (Sec. 4.1, cutPayoff): a new payoff in which
 * every payoff(t, p, q) is guarded as if(t + t0 < now, 0, payoff(t, p, q)),
 * so pricing it with opts.t_now = n counts only the cashflows on days >= n
 * (Thm. 5) without recompiling the contract.  ctx may be NULL. */
int pmc_payoff_cut(pmc_ctx* ctx, const pmc_payoff* in, pmc_payoff** out);

/* Device source of the compiled payoff engine for this payoff: the engine
 * kernel body plus the payoff expression translated to a HIP device function
 * (Sec. 6's code-generation route; compile with -DPMC_REAL=float|double
 * -DPMC_RNG=0|1 -DPMC_A=<assets> -DPMC_MEM=0|1, optionally -DPMC_P=<paths
 * per lane> -DPMC_FULL=<whole-path capacity> -DPMC_WAVES=<waves per SIMD>
 * -DPMC_SINGLE=1 (one instrument, fixed grid stride: no work queue or
 * instance order) -DPMC_OWN=1 (each block factors the correlation matrix
 * itself; generated paths only)).
 * tenv: NULL for the generic function (template values read per instance),
 * else the function generated for that template environment, as the engine
 * builds it for launches whose paths it holds whole (loopif iterations
 * written out, fixed reads; the generic one if that would be too large).
 * Copies at most cap bytes (NUL-terminated) to buf and stores the full
 * length (without NUL) in *len; buf may be NULL to query.  Returns
 * PMC_E_TENV for an invalid template environment. */
int pmc_payoff_source(const pmc_payoff* p, const int32_t* tenv, char* buf, size_t cap, size_t* len);

typedef struct pmc_payoff_info {
  int n_instr;      /* bytecode length */
  int n_regs;       /* registers per lane the interpreter uses */
  int loop_depth;   /* deepest loopif nesting */
  int n_time_exprs; /* distinct template expressions (folded per tenv) */
  int n_parties;    /* distinct party names */
  int n_assets;     /* model observables the payoff was loaded with */
  int n_params;     /* parameter observables */
  int n_tvars;      /* template variables */
} pmc_payoff_info;
int pmc_payoff_get_info(const pmc_payoff* p, pmc_payoff_info* out);

/* Simulated days for one template environment: the sorted distinct days > 0
 * that the expression can read for an asset (the re-indexed time grid of
 * the Futhark backend, Sec. 6.2; the horizon bound HOR of Sec. 4).
 * days_out may be NULL to query *n_slots only; else it must hold
 * max_days entries.  *horizon receives the largest day read (model or
 * payoff).  Errors: PMC_E_TENV, PMC_E_HORIZON. */
int pmc_payoff_grid(const pmc_payoff* p, const int32_t* tenv, int32_t* days_out, int max_days,
                    int* n_slots, int* horizon);

/* Whether, for this template environment and a simulation starting on day
 * sim_from (0, or the last day of a price history), the expression reads
 * the simulated days in non-decreasing order (checked with every branch and
 * loop iteration taken).  If so (*streams = 1), the compiled engine
 * generates its Philox paths as a stream: each date once, holding only the
 * newest prices, and may give each lane several paths.  Errors: PMC_E_TENV,
 * PMC_E_HORIZON. */
int pmc_payoff_streams(const pmc_payoff* p, const int32_t* tenv, int32_t sim_from, int* streams);

/* Risk-neutral GBM with constant rate, no dividends.  Prices S_a start at
 * spot[a]; log-price increments between simulated days are
 * (rate - vol_a^2/2) dt + vol_a sqrt(dt) w_a, w = L z, L L^T = corr,
 * dt = (day_s - day_{s-1}) * years_per_day.  Discount
 * d(day) = exp(-rate * day * years_per_day).  corr is n_assets x n_assets
 * row-major (NULL = identity). */
typedef struct pmc_gbm {
  int n_assets;
  const double* spot;
  const double* vol;
  const double* corr;
  double rate;
  double years_per_day;
} pmc_gbm;

typedef struct pmc_opts {
  uint64_t n_paths;        /* paths per price, 1 .. 2^32 */
  int rng;                 /* PMC_RNG_PHILOX or PMC_RNG_SOBOL */
  uint64_t seed;           /* Philox key = (seed mod 2^32, seed div 2^32) */
  uint32_t instance;       /* Philox counter word 2 (batched: per instance) */
  int precision;           /* PMC_FP32 (FP32 paths/payoffs, FP64 sums) or PMC_FP64 */
  int32_t t_now;           /* value of (now), the current time (Sec. 4.1) */
  const char* party_from;  /* flows party_from -> party_to count positive */
  const char* party_to;
  int mode;                /* PMC_MODE_*: fused (generate paths in registers),
                              two-phase (store SoA paths, then evaluate), auto */
  void* payoffs_dev;       /* optional: per-path payoff out, float[N] (FP32) or
                              double[N] (FP64); NULL to skip */
  int block;               /* threads per block, 0 = default (256) */
  int engine;              /* PMC_ENGINE_*: how the payoff runs on the device */
  /* Optional price history (Sec. 4.1: the environment is historical data up
   * to the current time and simulated data after it): history[a *
   * history_len + j] is the observed price of asset a on day t_now -
   * history_len + 1 + j, so the history ends on the current day t_now (>= 0).
   * A day up to t_now then reads the history (days before its first one read
   * its first price); the simulation starts on day t_now from the history's
   * last prices (model.spot is not used) and covers the days after it.  The
   * discount function stays d(day) = exp(-rate * day * years_per_day)
   * (Thm. 5).  NULL: days up to 0 read model.spot and the simulation starts
   * on day 0.  Host memory, read during the call; prices finite and > 0. */
  const double* history;
  int32_t history_len;
} pmc_opts;

typedef struct pmc_result {
  double price;       /* mean discounted payoff */
  double std_err;     /* sample SD (N-1) / sqrt(N) */
  double sum, sum_sq; /* FP64 sum and sum of squares over paths */
  uint64_t n_paths;
  uint64_t path_dates; /* n_paths * n_slots */
  int n_slots;
  int mode_used;
  double ms;          /* device time of the whole kernel sequence (HIP events) */
  double gen_ms;      /* two-phase only: path generation kernel */
  double eval_ms;     /* the Monte Carlo / payoff kernel (fused single pricing:
                         from the start marker to the pricing kernel's end,
                         before the one-block finishing reduction; two-phase:
                         the evaluator and its reduction) */
  int engine_used;    /* PMC_ENGINE_INTERPRETER or PMC_ENGINE_COMPILED */
} pmc_result;

/* Price one instrument: tenv[n_tvars] (naturals), params[n_params].
 * Random words: Philox word w = slot*A + asset of path p is element w%4 of
 * the block with counter (p, w/4, instance, 0); Sobol dimension w, point p
 * (unscrambled, Joe-Kuo, Gray order).  Uniforms: FP64 (x+0.5)2^-32, FP32
 * (x>>9 + 0.5)2^-23; normals by inverse CDF (AS241).
 * Errors: PMC_E_ARG, PMC_E_TENV, PMC_E_HORIZON, PMC_E_NOT_PD, PMC_E_HIP,
 * PMC_E_OOM. */
int pmc_price(pmc_ctx* ctx, const pmc_payoff* p, const int32_t* tenv, const double* params,
              const pmc_gbm* model, const pmc_opts* opts, pmc_result* out);

/* Allocation-free variant of pmc_price, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, checks, random streams
 * and result as pmc_price with opts.engine = PMC_ENGINE_INTERPRETER and
 * opts.mode = PMC_MODE_FUSED: the same kernels and grid, so the same sums
 * bit for bit.  The call allocates no device or pinned memory: its tables,
 * per-block partials, factorisation status and result live in a static
 * device array of 4 MiB + 256 bytes per GPU (held until the process ends;
 * its address is looked up when a context is created), and its uploads and
 * result copy use pageable host memory.  Every call on one GPU shares that
 * array and leaves its contents behind; calls that overlap on one GPU (other
 * threads, contexts or streams) race and must not be made.  opts.payoffs_dev
 * works as in pmc_price.
 * Errors: those of pmc_price; PMC_E_UNSUPPORTED for opts.mode =
 * PMC_MODE_TWO_PHASE, opts.engine = PMC_ENGINE_COMPILED (run-time compiled
 * code is loaded into newly allocated memory), or tables (bytecode, time and
 * discount tables, Sobol direction numbers) beyond the array's 2 MiB table
 * area (e.g. Sobol with more than about 16,000 dimensions); PMC_E_HIP if the
 * array's address could not be looked up on this device. */
int pmc_price_noalloc(pmc_ctx* ctx, const pmc_payoff* p, const int32_t* tenv, const double* params,
                      const pmc_gbm* model, const pmc_opts* opts, pmc_result* out);

/* Batch of instances of one loaded payoff (templated instruments priced
 * with different template values and parameters, Sec. 2 and Sec. 6.2),
 * run as one persistent launch over (instance, path-tile) work items taken
 * longest-first from an atomic queue, replayed from a captured HIP graph.
 * tenv: n_inst x n_tvars; params: n_inst x n_params.  If per_instance_model
 * is nonzero, spot/vol are n_inst x A and corr n_inst x A x A (each factored
 * on the device); else the shared model's arrays are used.  instance_ids
 * (optional) give each instance's Philox counter word 2 (default: its
 * index).  out[n_inst].  The opts.payoffs_dev output is not supported here. */
typedef struct pmc_batch {
  int n_inst;
  const int32_t* tenv;
  const double* params;
  int per_instance_model;
  const double* spot;
  const double* vol;
  const double* corr;
  const uint32_t* instance_ids;
} pmc_batch;
int pmc_price_batch(pmc_ctx* ctx, const pmc_payoff* p, const pmc_batch* batch,
                    const pmc_gbm* model, const pmc_opts* opts, pmc_result* out);

/* Autotune the batched launch for this payoff and batch by timing graph
 * replays of every candidate tile: threads per block (64, 128, 256), rounds
 * per thread (1, 2, 4) and paths per lane per round (1, or 2 where the batch
 * streams its paths: compiled engine, Philox, every instance's expression
 * reading its dates strictly forward).  The choice is kept in the context
 * and, when cache_path is not NULL, appended to that text file as a line
 * "key block ppt lanes" (key = device, payoff hash, batch shape) and reused
 * from it on later calls (a line that is not a launchable tile is ignored).
 * *block_out, *ppt_out and *lanes_out (each may be NULL) receive it. */
int pmc_autotune_batch(pmc_ctx* ctx, const pmc_payoff* p, const pmc_batch* batch,
                       const pmc_gbm* model, const pmc_opts* opts, const char* cache_path,
                       int* block_out, int* ppt_out, int* lanes_out);

/* Bump-and-revalue risk over a batch (the risk runs of thousands of
 * pricings of one compiled contract that motivate the engine, end of Sec. 6.2).
 * For every instance of the batch (same layout and model rules as
 * pmc_price_batch) the library prices 1 + 4A scenarios: the base model, then
 * for each asset a the spots S_a + h_a and S_a - h_a (h_a = rel_spot_bump *
 * S_a), then for each asset the volatilities sigma_a + k and sigma_a - k
 * (k = abs_vol_bump).  All scenarios of an instance use the instance's random
 * stream (common random numbers) and run as one persistent batch launch.
 * Central differences give delta_a = (V+ - V-) / 2h_a, gamma_a =
 * (V+ - 2V + V-) / h_a^2 and vega_a = (V+ - V-) / 2k.  out[n_inst]; entries
 * beyond A are zero; ms is the device time of the whole launch.
 * Errors: those of pmc_price_batch; PMC_E_ARG if 0 < rel_spot_bump < 1 and
 * 0 < abs_vol_bump < sigma_a do not hold; PMC_E_UNSUPPORTED with a price
 * history (opts.history: the simulation would not start from the spots). */
typedef struct pmc_risk_opts {
  double rel_spot_bump;
  double abs_vol_bump;
} pmc_risk_opts;
typedef struct pmc_greeks {
  double price, std_err;
  double delta[PMC_MAX_ASSETS];
  double gamma[PMC_MAX_ASSETS];
  double vega[PMC_MAX_ASSETS];
  double ms;
} pmc_greeks;
int pmc_risk_batch(pmc_ctx* ctx, const pmc_payoff* p, const pmc_batch* batch, const pmc_gbm* model,
                   const pmc_opts* opts, const pmc_risk_opts* risk, pmc_greeks* out);

/* Parity hooks.  pmc_gen_paths writes the simulated prices S[slot][asset][path]
 * (float or double by opts.precision) to paths_dev, and optionally the raw
 * random words [word][path] (uint32) to words_dev and the normals
 * [word][path] to normals_dev (same float type).  pmc_eval_paths evaluates
 * the payoff on caller-supplied prices in that layout, writing per-path
 * payoffs to opts.payoffs_dev (may be NULL) and the sums to *out. */
int pmc_gen_paths(pmc_ctx* ctx, const pmc_payoff* p, const int32_t* tenv, const pmc_gbm* model,
                  const pmc_opts* opts, void* paths_dev, uint32_t* words_dev, void* normals_dev);
int pmc_eval_paths(pmc_ctx* ctx, const pmc_payoff* p, const int32_t* tenv, const double* params,
                   const pmc_gbm* model, const pmc_opts* opts, const void* paths_dev,
                   pmc_result* out);

/* Lower Cholesky factors of n row-major m x m matrices, computed on the
 * device in FP64 (the factor every price call uses).  Host in/out.
 * Errors: PMC_E_NOT_PD (first failing matrix index in pmc_last_error). */
int pmc_cholesky(pmc_ctx* ctx, const double* a, int n, int m, double* l_out);

/* Peak-rate probe (diagnostic, for roofline figures): the vector-ALU lane
 * operations per second this device sustains for one instruction class,
 * from a kernel of independent dependency chains on 2048 blocks of 256
 * threads (8 waves per SIMD on 256 CUs) with no memory traffic in its timed
 * loop.  kind 0: FP32 fused multiply-add (v_fma_f32); 1: 32-bit xor and add;
 * 2: 32 x 32 -> 64-bit multiply-add (v_mad_u64_u32) and a 32-bit add;
 * 3: FP32 exp2 (v_exp_f32) and a multiply; 4: independent FP32 FMA and
 * 32-bit xor chains interleaved.  Allocates and frees 32 bytes. */
int pmc_probe_valu(pmc_ctx* ctx, int kind, double* lane_ops_per_s);

/* ---- learned surrogate: MLP 8 -> W -> W -> W -> 1 (GELU), BF16 weights and
 * activations with FP32 accumulation on MFMA; FP32 master weights and Adam.
 * Inputs are min-max scaled to [-1, 1] by the library (lo/hi per input);
 * the network predicts price / y_scale. */
typedef struct pmc_mlp pmc_mlp;
int pmc_mlp_create(pmc_ctx* ctx, int n_in, int width, uint64_t seed, const double* in_lo,
                   const double* in_hi, double y_scale, pmc_mlp** out);
void pmc_mlp_free(pmc_mlp* m);
/* Number of parameters (weights and biases of all layers). */
/* Save the network (shape, input box, y_scale and FP32 master weights) to a
 * binary file; pmc_mlp_load re-creates it on ctx's device with fresh Adam
 * state.  The network's activation is the tanh form of GELU (file format
 * 2; files of format 1, whose networks used the erf form, are refused).
 * Errors: PMC_E_ARG (file cannot be opened or written), PMC_E_PARSE (not a
 * file written by pmc_mlp_save of this format and a supported shape). */
int pmc_mlp_save(const pmc_mlp* m, const char* path);
int pmc_mlp_load(pmc_ctx* ctx, const char* path, pmc_mlp** out);
int64_t pmc_mlp_num_params(const pmc_mlp* m);
/* Host FP32 copies of the master weights in the order W1 b1 W2 b2 W3 b3 W4 b4,
 * each W row-major [out][in]. */
int pmc_mlp_get_params(const pmc_mlp* m, float* out);
int pmc_mlp_set_params(pmc_mlp* m, const float* in);
typedef struct pmc_train_opts {
  int batch;          /* samples per Adam step */
  double lr_max, lr_min; /* cosine schedule from lr_max to lr_min over total_steps */
  int64_t total_steps;
  double beta1, beta2, eps;
  int eager;          /* 0: steps replayed from a captured graph of 16 steps;
                         1: the same kernels launched one by one (same results) */
} pmc_train_opts;
/* One pass over n samples (x_dev [n][n_in] float, raw inputs; y_dev [n]
 * float prices) in order, one Adam step per full batch (a trailing partial
 * batch is skipped); *mean_loss receives the mean squared error of the
 * scaled target over the pass.  o->batch must be a multiple of 64.  A step
 * (forward, loss, gradients, Adam with the BF16 repack of the weights: 6
 * launches) is captured 16 times in a row as one HIP graph per batch size,
 * replayed for every 16 steps (the steps left over in a pass are launched
 * one by one); the batch position, learning rate and bias corrections are
 * read from a device-side step record written at the start of the pass, so
 * x_dev and y_dev may change between passes without a new capture.  The
 * call returns after the pass has finished on the device. */
int pmc_mlp_train_epoch(pmc_mlp* m, const float* x_dev, const float* y_dev, int64_t n,
                        const pmc_train_opts* o, double* mean_loss);
/* Forward pass: y_dev[n] prices (float) for raw inputs x_dev[n][n_in].
 * The work is enqueued on the context's stream and the call returns once
 * it is launched, like a kernel launch: y_dev is ready when that stream
 * reaches this point (order later work on the same stream, or synchronize
 * it, before reading y_dev; x_dev must stay valid until then). */
int pmc_mlp_infer(pmc_mlp* m, const float* x_dev, float* y_dev, int64_t n);
/* Prices from the surrogate with Monte Carlo as the fallback: point i, with
 * raw inputs x[i][n_in] (host memory), is priced by the network when every
 * input lies in the network's input box [lo, hi] (the box it was created
 * with, which its training data covers), and otherwise by Monte Carlo:
 * instance i of `batch` (n_inst = n, in the same order; the same layout and
 * rules as pmc_price_batch) priced with payoff p, `model` and `opts`, all
 * out-of-box instances in one pmc_price_batch launch.  An instance keeps its
 * stream id (batch->instance_ids[i], else i), so a fallback price equals the
 * one pmc_price_batch gives that instance within any batch.  price_out[n];
 * std_err_out[n] (optional) receives the Monte Carlo standard error, 0 for a
 * network price; route_out[n] (optional) 0 for the network, 1 for Monte
 * Carlo.  Errors: PMC_E_ARG (n_inst != n, missing arrays), and those of
 * pmc_mlp_infer and pmc_price_batch. */
int pmc_mlp_price(pmc_mlp* m, const double* x, int64_t n, const pmc_payoff* p, const pmc_batch* batch,
                  const pmc_gbm* model, const pmc_opts* opts, double* price_out, double* std_err_out,
                  int* route_out);
/* Loss and gradients of the mean squared error over n samples (1 <= n <=
 * 65536) at the current weights (FP32 gradients, host out, same order as
 * get_params). */
int pmc_mlp_loss_grad(pmc_mlp* m, const float* x_dev, const float* y_dev, int64_t n,
                      double* loss, float* grad_out);

#ifdef __cplusplus
}
#endif
#endif /* PMC_H_ */

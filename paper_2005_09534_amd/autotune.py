"""Autotuner of the POLFED hot path on one GPU.

Two choices are tuned, both through the C ABI of libpolfed:

* the launch shape of the fused Chebyshev-step kernel (threads per group,
  16-byte loads per lane, persistent groups per CU, rank tables in LDS,
  streamed loads before or after the neighbour gathers, neighbour ranks from
  the tables, incrementally or from the stored pattern, column slices across
  the XCDs) for a (chain
  length L, block width,
  precision): each candidate applies the filter for a few dozen steps to a
  random block of the chain and is timed with the library's HIP-event
  counters; the fastest shape per HBM-second wins
  (``polfed_set_step_shape``);
* the filter recurrence (Clenshaw or the forward form, ``tune_form``): the
  same filter applied both ways, the shorter time wins
  (``polfed_set_filter_form``);
* the Lanczos block size for (L, precision, N_ev): a sample of realisations
  (one, or a batch of a few of the same L) is solved with each candidate
  width and the shortest time to N_ev per realisation wins
  (``polfed_set_block_size``).

Results are cached as JSON (default: $POLFED_TUNE_CACHE, else
~/.cache/polfed_tune.json) keyed by "shape:L:J2nonzero:precision:width" and
"block:L:J2nonzero:precision:nev", and re-applied by ``apply_cache``.
"""

import itertools
import json
import os
import time

# (threads, 16-byte loads per lane, groups per CU, LDS rank tables, streamed
# loads issued before the gathers, incremental neighbour ranks, XCD column
# slices)
LAUNCH = [(t, lpl, wpc) for t, lpl, wpc in
          itertools.product((256, 512, 1024), (1, 2, 4), (1, 2, 4, 8, 16))
          if wpc * t <= 2048]
# (rank mode 2, the stored pattern, stages no tables: lds = 0 only)
SHAPES = [(t, lpl, wpc, lds, early, ranki, xcd)
          for (t, lpl, wpc), lds, early, ranki, xcd in
          itertools.product(LAUNCH, (1, 0), (0, 1), (0, 1, 2), (1, 2, 4, 8))
          if not (ranki == 2 and lds == 1)]


def cache_path():
    return os.environ.get("POLFED_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "polfed_tune.json"))


def load_cache(path=None):
    path = path or cache_path()
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def _key(kind, L, J2, precision, x):
    return f"{kind}:{L}:{int(J2 != 0.0)}:{precision}:{x}"


def staged_candidates(best, width):
    """Second stage of the default search: the launch shapes (threads, loads
    per lane, groups per CU) with every column-slice count that splits the
    width, the other fields as in `best`."""
    return [(t, lpl, wpc) + tuple(best[3:6]) + (xcd,)
            for (t, lpl, wpc) in LAUNCH for xcd in (2, 4, 8) if xcd <= width]


def tune_shape(ctx, chain, width, precision, steps=None, shapes=None, cache=None, margin=0.03):
    """Fastest step-kernel shape for the chain's L at this width/precision.

    With `shapes` given, every candidate in it is timed.  By default the
    search has two stages: every unsliced shape, then the launch shapes with
    2, 4 and 8 column slices around the best of the first stage.  The shape
    in force (the library default, or an earlier choice) is kept unless
    another is faster by more than `margin`, so that near-ties do not flip
    the choice from run to run.  Leaves the choice set on ctx; returns
    (shape, GB/s)."""
    import torch
    from . import polfed as pf
    m = pf.make_model(chain.L, chain.J1, chain.J2, chain.Delta, chain.h)
    n = pf.dim(chain.L)
    dt = torch.float32 if precision else torch.float64
    X = torch.randn((n, width), device="cuda", dtype=torch.float64).to(dt)
    Y = torch.empty_like(X)
    if steps is None:
        steps = max(8, min(200, int(2e9 / (n * width * (4 if precision else 8) * 4))))
    E0, E1 = -2.0 * chain.L, 2.0 * chain.L  # any enclosing interval; cost is independent of it

    def rate(sh):
        ctx.set_step_shape(chain.L, width, precision, *sh)
        ctx.apply_filter(m, E0, E1, 0.0, 2, X, out=Y)
        ctx.filter_stats(reset=True)
        ctx.apply_filter(m, E0, E1, 0.0, steps, X, out=Y)
        st = ctx.filter_stats(reset=True)
        return st["bytes"] / st["gpu_s"] / 1e9

    current = tuple(ctx.get_step_shape(chain.L, width, precision))
    best = (current, rate(current))
    seen = {current}

    def search(cands):
        nonlocal best
        for sh in cands:
            sh = tuple(sh)
            if sh in seen:
                continue
            seen.add(sh)
            gbs = rate(sh)
            if gbs > best[1] * (1.0 + margin if best[0] == current else 1.0):
                best = (sh, gbs)

    if shapes is not None:
        search(shapes)
    else:
        search([sh for sh in SHAPES if sh[6] == 1])
        search(staged_candidates(best[0], width))
    ctx.set_step_shape(chain.L, width, precision, *best[0])
    if cache is not None:
        cache[_key("shape", chain.L, chain.J2, precision, width)] = list(best[0]) + [best[1]]
    return best


def tune_form(ctx, chain, width, precision, K=None, margin=0.03):
    """Filter recurrence with the shorter time for one filter application of
    order K on this chain and width (step shape as set).  Clenshaw is kept
    unless the forward form is faster by more than `margin`.  Leaves the
    choice set on ctx; returns (form, {form: seconds})."""
    import torch
    from . import polfed as pf
    m = pf.make_model(chain.L, chain.J1, chain.J2, chain.Delta, chain.h)
    n = pf.dim(chain.L)
    dt = torch.float32 if precision else torch.float64
    X = torch.randn((n, width), device="cuda", dtype=torch.float64).to(dt)
    Y = torch.empty_like(X)
    if K is None:
        K = max(8, min(200, int(2e9 / (n * width * (4 if precision else 8) * 4))))
    E0, E1 = -2.0 * chain.L, 2.0 * chain.L
    secs = {}
    for form in (pf.FORM_CLENSHAW, pf.FORM_FORWARD):
        ctx.set_filter_form(form)
        ctx.apply_filter(m, E0, E1, 0.0, K, X, out=Y)  # warm (graph capture)
        ctx.filter_stats(reset=True)
        ctx.apply_filter(m, E0, E1, 0.0, K, X, out=Y)
        secs[form] = ctx.filter_stats(reset=True)["gpu_s"]
    form = (pf.FORM_FORWARD if secs[pf.FORM_FORWARD] * (1.0 + margin) < secs[pf.FORM_CLENSHAW]
            else pf.FORM_CLENSHAW)
    ctx.set_filter_form(form)
    return form, secs


def tune_block(ctx, chains, nev, precision, widths=(4, 8, 16, 32), cache=None, shape_cache=None):
    """Block size with the shortest time to nev per realisation.

    `chains` is one chain or a list of chains of one length L: a list is
    solved as one batch (polfed_solve_batch), so the choice reflects batch
    throughput rather than the latency of a single solve.  Tunes the step
    shape of each width first.  Leaves the choice set on ctx; returns
    (block, seconds per realisation) or None when no width converged."""
    import torch
    from . import polfed as pf
    if not isinstance(chains, (list, tuple)):
        chains = [chains]
    L = chains[0].L
    if any(c.L != L for c in chains):
        raise ValueError("tune_block: chains of one length only")
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    best = None
    times = {}
    for s in widths:
        if s > nev:  # wider blocks than N_ev waste columns and can hit the column cap
            continue
        if len(models) == 1:
            tune_shape(ctx, chains[0], s, precision, cache=shape_cache)

        def run():
            if len(models) == 1:
                r = ctx.solve(models[0], nev, block_size=s, precision=precision, vectors=False)
                return [r["status"]]
            return ctx.solve_batch(models, nev, block_size=s, precision=precision,
                                   vectors=False)["status"]

        def timed():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = run()
            torch.cuda.synchronize()
            return st, (time.perf_counter() - t0) / len(models)
        run()  # warm (graph capture, buffers)
        st, t = timed()
        if len(models) > 1:
            # the batched kernel has shapes of its own (a launch walks many
            # realisations; a single chain's tuned shape, chosen where a
            # launch is short, can be far off there): re-time the
            # groups-per-CU choice of the batch shape on the sample batch,
            # keep a change only when it gains more than 3%
            base = tuple(ctx.get_batch_shape(L, s, precision))
            best_sh, best_st, best_t = base, st, t
            for wpc in (2, 4, 8, 16):
                sh = (base[0], base[1], wpc) + base[3:]
                if wpc == base[2] or wpc * base[0] > 2048:
                    continue
                ctx.set_batch_shape(L, s, precision, *sh)
                run()
                st_w, t_w = timed()
                if all(x == pf.OK for x in st_w) and t_w < best_t * 0.97:
                    best_sh, best_st, best_t = sh, st_w, t_w
            ctx.set_batch_shape(L, s, precision, *best_sh)
            if shape_cache is not None and best_sh != base:
                shape_cache[_key("bshape", L, chains[0].J2, precision, s)] = list(best_sh) + [0.0]
            st, t = best_st, best_t
        if all(x == pf.OK for x in st):
            times[s] = t
            if best is None or t < best[1]:
                best = (s, t)
    if best is not None and len(models) > 1:
        # a full batch keeps the device busy even with narrow blocks, which a
        # small sample does not show: among widths within 10% of the best
        # sample time, take the narrowest (fewest Lanczos columns); at L=18
        # with 170 realisations s=4 measured 89 s against 98 s for s=8, which
        # the 8-member sample had put 4% apart
        s_min = min(w for w, t in times.items() if t <= 1.10 * best[1])
        best = (s_min, times[s_min])
    if best is not None:
        ctx.set_block_size(L, precision, nev, best[0])
        if cache is not None:
            cache[_key("block", L, chains[0].J2, precision, nev)] = [best[0], best[1]]
    return best


def apply_cache(ctx, cache):
    """Set every cached shape and block size on ctx."""
    for k, v in cache.items():
        kind, L, _j2, prec, x = k.split(":")
        if kind == "shape":
            # entries are the shape followed by its GB/s; older ones lack the
            # rank-mode field (tables then) and the column slices (none)
            sh = [int(t) for t in v[:-1]]
            sh = (sh + [0, 1][len(sh) - 5:])[:7]
            ctx.set_step_shape(int(L), int(x), int(prec), *sh)
        elif kind == "bshape":
            ctx.set_batch_shape(int(L), int(x), int(prec), *[int(t) for t in v[:-1]])
        elif kind == "block":
            ctx.set_block_size(int(L), int(prec), int(x), int(v[0]))

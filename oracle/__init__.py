"""OASM oracle -- test infrastructure only (see oracle.py and oasm_oracle.c)."""
from .oracle import (  # noqa: F401
    FilterResult,
    PairResult,
    build,
    filter_hits,
    hset_all,
    hset_at_ends,
    lev,
    levcalc,
    levcalc_many,
    raw_hits,
    run_pair,
    run_pairs,
    sellers_column,
)

"""Throughput and scaling figures as the paper reports them.

Speedup and efficiency follow the results table of section 5 (Results and
Analysis): speedup = T1 / Tp, efficiency = 100 * speedup / p.  The sequential
figure of Table 1 (section 3.1) is the mean of ten runs.
"""
from __future__ import annotations


def speedup(t1: float, tp: float) -> float:
    return float(t1) / float(tp)


def efficiency(t1: float, tp: float, p: int) -> float:
    """Parallel efficiency in percent."""
    return 100.0 * speedup(t1, tp) / float(p)


def mean(xs) -> float:
    xs = [float(x) for x in xs]
    return sum(xs) / len(xs)


def mwords_per_s(words: int, seconds: float) -> float:
    return float(words) / float(seconds) / 1e6

"""Outcome codes of a solve (oracle; test infrastructure only).

The paper distinguishes converged runs from runs that diverge ("-") or
stagnate above the requested accuracy ("- [x]") in its tables (Section 5.2).
"""
import enum


class Outcome(enum.IntEnum):
    CONVERGED = 0
    STAGNATED = 1
    DIVERGED = 2
    BREAKDOWN = 3
    MAX_ITER = 4

"""Shared test helpers (test infrastructure): the parity metric lives in the package's metrics
module, where bench.py reads it too."""
from paper_2410_03632_amd.metrics import g16_err  # noqa: F401

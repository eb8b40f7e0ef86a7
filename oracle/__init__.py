"""FP64 CPU oracle -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the HIP library and never imports it.
Every function names the passage of Burden, Percival & Howlett (arXiv:1504.02591)
it follows.  Functions whose result no independent pin fixes are marked
"parity unpinned" in their docstring.
"""
from . import recon_oracle  # noqa: F401

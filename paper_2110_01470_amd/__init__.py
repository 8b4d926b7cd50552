"""MI355X-native Simplified Swarm Optimization (arXiv 2110.01470).

The optimiser runs in hand-written HIP kernels behind the C ABI of
``include/sso.h`` (``libsso.so``); ``binding`` is the thin ctypes layer over
it and ``inputs`` draws the seeded synthetic workloads.  Importing this
package loads nothing; ``from paper_2110_01470_amd.binding import Swarm``
loads the library and fails loudly when it has not been built.
"""

__all__ = ["binding", "inputs"]

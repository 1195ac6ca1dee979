"""MI355X-native explicit particle-in-cell cycle (cubic gather, Boris push,
charge-conserving cubic deposit, Yee / perfect-dispersion FDTD).

The compute path is the HIP library ``libpic355.so`` built from ``csrc/``;
``paper_1204_0838_amd.pic`` is its thin ctypes binding.  Nothing is loaded at
import time so that the input generator can be used on hosts without a GPU.
"""

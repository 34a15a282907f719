"""MI355X (gfx950) PAGD solver for fully implicit PFC / FCH steps.

The compute path is the HIP library ``libpfch.so`` (sources in ``csrc/``,
C ABI in ``include/pfch.h``); ``pfch`` is its thin ctypes binding.
"""

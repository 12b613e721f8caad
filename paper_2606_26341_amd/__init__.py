"""hipipm: batched primal-dual interior-point NLP solver for one AMD Instinct MI355X (gfx950).

The solver itself is the HIP library ``libhipipm.so`` behind the C ABI declared in
``include/hipipm.h``; ``paper_2606_26341_amd.hipipm`` is its thin ctypes binding.
Importing this package loads nothing.
"""

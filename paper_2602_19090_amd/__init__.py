"""MI355X (gfx950) eigenvector refinement: Ogita-Aishima iterations with
Ozaki-scheme INT8 slice products (Terao & Ozaki, arXiv 2602.19090).

The compute path is the HIP library ``librefeig.so`` (C ABI in
``include/refeig.h``); ``paper_2602_19090_amd.binding`` is its ctypes binding.
"""

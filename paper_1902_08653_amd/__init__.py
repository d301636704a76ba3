"""MI355X (gfx950) coordinate-descent data detection and precoding for massive MU-MIMO.

Decentralized coordinate-descent detection (Algorithm 1) and precoding
(Algorithm 2) of Li, Castaneda, Jeon, Cavallaro and Studer (arXiv 1902.08653),
as hand-written HIP kernels behind the C ABI of ``include/cdm.h``.

Modules: ``cdm`` (the binding), ``inputs`` (seeded synthetic workloads),
``build`` (hipcc build of ``libcdm.so``).
"""

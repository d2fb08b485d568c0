"""MI355X-native differentiable Gaussian rasterizer for Gaussian-SLAM (arXiv 2312.10070).

The compute path is the C-ABI library ``libgsr.so`` (hand-written HIP for
gfx950, declared in ``include/gsr.h``); :mod:`paper_2312_10070_amd.gsr` is its
thin ctypes binding and :mod:`paper_2312_10070_amd.render` wraps it in
``torch.autograd.Function``. :mod:`paper_2312_10070_amd.synth` only generates
seeded inputs. Importing this package does not load the library; the first
call that needs it does, and raises if it is missing.
"""

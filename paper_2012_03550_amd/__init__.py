"""SGD_Tucker minibatch update on MI355X (gfx950).

The compute path is the HIP library ``libstdecomp.so`` (C ABI declared in
``include/stdecomp.h``); :mod:`paper_2012_03550_amd.binding` is its thin
ctypes front end.  :mod:`paper_2012_03550_amd.synth` draws seeded synthetic
workloads.
"""

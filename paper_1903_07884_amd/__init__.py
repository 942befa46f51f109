"""MI355X (gfx950) voxel VIE solver with Chan-Olkin circulant preconditioning.

The solver lives in the HIP library ``libvie.so`` (C ABI in include/vie.h);
``vie`` is its Python binding and ``workloads`` builds seeded synthetic inputs.
"""

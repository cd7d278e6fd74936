"""Seeded synthetic inputs shared by the checkpoint path and its oracle.

This package only *generates* memory images and scenario descriptions; it
holds none of the checkpoint arithmetic (no diff, compaction, CRC or image
format).  Three implementations of the same counter-based byte generator live
here and are cross-checked by tests:

* ``csrc/synth_host.c``  -- host C (used to regenerate inputs for the oracle),
* ``csrc/synth_dev.hip`` -- HIP kernels (used to fill device memory),
* :func:`splitmix_words` -- numpy (the plain reference for both).

Scenario choices (page sets, sizes, runs, residency) come from
``numpy.random.Generator(PCG64(seed))`` in :mod:`synth.scenarios`.
"""
from .lib import (  # noqa: F401
    build,
    host_lib,
    dev_lib,
    splitmix_words,
    fill_host,
    mutate_host,
    fill_dev,
    mutate_dev,
    saxpy_loop_dev,
    copy_dev,
    read2_dev,
    mutate_frac_dev,
    clobber_frac_dev,
)

"""Seeded synthetic echelle workloads (inputs only).

This package builds the inputs that both the FP64 oracle and the GPU library
consume: detector geometry, per-trace spectral-format polynomials, PSF tables
and input spectra.  It contains none of the rendering arithmetic: it never
maps a wavelength to the detector, never integrates a PSF over a pixel and
never accumulates a frame.
"""
from .synth import (Trace, Psf, Scene, Request, scene, request, SCENES,
                    CONFIG_NOTES, detector_frame, prnu_map, XTALK_CCD)

__all__ = ["Trace", "Psf", "Scene", "Request", "scene", "request", "SCENES",
           "CONFIG_NOTES", "detector_frame", "prnu_map", "XTALK_CCD"]

"""Unbinned maximum-likelihood fits on AMD MI355X (gfx950).

The hot path of the MoreFit method: the negative log-likelihood
-sum_i w_i ln P(x_i|theta) of a model built from a catalogue of PDFs, with
its analytic gradient and Hessian, evaluated by hand-written HIP kernels
behind a C ABI (include/uml.h, libuml.so).  This package holds the kernels'
sources (csrc/), their build script and a ctypes binding (uml.py).
"""
from .uml import (Data, Model, UmlError, lib, uml_eval_hessian, uml_eval_nll,  # noqa: F401
                  uml_eval_nll_grad, uml_eval_nll_grad_dev, uml_fit, uml_fit_batch, uml_version)

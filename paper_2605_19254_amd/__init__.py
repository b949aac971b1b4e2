"""MI355X-native exact multi-modular (RNS) integer matrix product and a
Smith-form driver built on it.

The computation lives in librns.so (HIP kernels for gfx950 behind the C ABI of
include/rns.h); ``binding`` marshals torch device tensors into it.  Importing
the binding without the built library raises ImportError: there is no CPU
fallback.
"""
from .binding import (Context, GemmPlan, GemmProblem, MatmulPlan, MatmulProblem,  # noqa: F401
                      RnsError, Server, SmithResult, autotune, server_footprint, crt_reconstruct, modmatmul_batched,
                      lift_step, modmatmul_batched_noalloc, noalloc_scratch_bytes, base_convert,
                      rns_primes_below, rns_reduce, rns_reduce_mw, rns_strerror, smith_form, largest_invariant, words_to_ints,
                      smith_massager, MassagerResult, unimodular_certify, UnimodularResult,
                      workspace_bytes)

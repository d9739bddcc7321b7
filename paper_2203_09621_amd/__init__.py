"""MI355X (gfx950) DNN-SP2-PT: zeroth- and first-order density matrices by a deep
layered network of SP2 steps, with hand-written HIP kernels behind a C ABI
(include/dmpt.h).  Python only marshals arguments; the HIP library does the work
and must be built (``python -m paper_2203_09621_amd.build``).  The library is
loaded on first use of any entry point; a missing library raises ImportError."""

_API = ("EXPORTS", "PRECISION", "DmptError", "dmpt_adjoint", "dmpt_batch_destroy",
        "dmpt_batch_info", "dmpt_batch_init", "dmpt_batch_response", "dmpt_congruence",
        "dmpt_contract", "dmpt_contract_noalloc", "dmpt_cpscf", "dmpt_inverse_factor", "solve_nonorth",
        "dmpt_destroy",
        "dmpt_gershgorin",
        "dmpt_init", "dmpt_layer_products", "dmpt_layer_trace", "dmpt_plan_rounds", "dmpt_plan_layer",
        "dmpt_probe_mfma",
        "dmpt_response", "dmpt_response2",
        "dmpt_selftest_mfma",
        "dmpt_set_hamiltonian", "response_function", "density_function",
        "dmpt_response_adjoint", "solve")


def __getattr__(name):
    if name in _API:
        from . import _native
        return getattr(_native, name)
    raise AttributeError(name)


__all__ = list(_API)

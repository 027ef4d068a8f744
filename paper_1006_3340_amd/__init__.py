"""MI355X Monte Carlo engine for the Lévy LIBOR model (Papapantoleon & Skovmand).

The computation lives in the HIP library ``liblll.so`` behind the C ABI of
``include/lll.h``; this package is its thin Python binding.  Importing the
package does not load the library; the first call does, and raises if the
library is missing.
"""
from ._lib import (EXACT, FIRST_ORDER, FP32, FP64, FROZEN, FULL, MLP_DRIFT, N_MAX,  # noqa: F401
                   N_MAX_EXACT, N_MAX_MP, PICARD, PICARD_MP, SECOND_ORDER,
                   Batch, LLLError, Mlp, Plan, caplet_greeks, load, philox, price_caplets,
                   sampler_math,
                   price_caplets_batched, price_caplets_static, fp32_fma_peak, fp32_mix_peak,
                   fp32_mfma_peak, version)

SCHEMES = {"full": FULL, "picard": PICARD, "frozen": FROZEN, "first_order": FIRST_ORDER,
           "second_order": SECOND_ORDER, "picard_mp": PICARD_MP, "exact": EXACT,
           "mlp_drift": MLP_DRIFT}

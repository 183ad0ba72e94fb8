"""MI355X-native batched GW log-likelihood, adjoint gradient, NUTS and SMC kernels."""

"""MI355X-native periodic adjoint (arXiv:1512.00616): HIP library binding."""

"""MI355X-native Hawkes log-likelihood + gradient (arXiv 2010.02994 hot path)."""

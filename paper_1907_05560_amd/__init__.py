"""MI355X-native bulb-model neutrino flavor evolution (XFLAT hot path)."""

"""MI355X-native short-characteristics radiative transfer (Davis, Stone & Jiang 2012)."""

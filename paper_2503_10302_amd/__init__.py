"""MI355X-native spin-glass Monte Carlo library (APT+ICM and DT-SQA hot path)."""

"""rtssa: next-reaction random-time stochastic simulation on AMD MI355X.
The HIP library is loaded on first use; see ``api``."""

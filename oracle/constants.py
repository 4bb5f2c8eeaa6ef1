"""Physical constants (CODATA 2018).  The paper uses e0, eps0, k_B, m_e without
giving values (Sec. 2, Poisson equation; Sec. 2.1, gas density)."""
E0 = 1.602176634e-19          # elementary charge [C]
EPS0 = 8.8541878128e-12       # vacuum permittivity [F/m]
KB = 1.380649e-23             # Boltzmann constant [J/K]
ME = 9.1093837015e-31         # electron mass [kg]
AMU = 1.66053906660e-27       # atomic mass unit [kg]

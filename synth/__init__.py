from .water import *  # noqa
